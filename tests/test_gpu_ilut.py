"""GPU parity of the ILUT(p, tol) local solvers (the RAS parameters' ILUT
solver with ilut_p and ilut_tol) for 3x3-block matrices, through the C ABI,
against the oracle's ILUT: the whole grid as one subdomain (type BILU0) and
RAS with ILUT local solves, applied per entry within 1e-12 of the largest
entry (times the amplification max|z|/max|r| on the literal reading; a
single drop or keep decision taken differently would move entries by about
tol x the row norm, far above that bar, so this also checks that the
device keeps exactly the oracle's blocks); GMRES(30) + RAS(ILUT)
solves against the oracle's; the error paths."""
import sys

import numpy as np
import pytest

torch = pytest.importorskip("torch")

from paper_1602_05901_amd import inputs as I  # noqa: E402
import oracle as O  # noqa: E402
from oracle import cpr as OC  # noqa: E402

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


def sysm(rsv, ctx, dims, seed=0, shift=2.0, sigma=1.0):
    cfg = I.GenConfig(*dims, I.LNK_IID, sigma, 0.0, shift, 0, 1e3, 1.0, seed)
    B = I.blocks(cfg)
    g = rsv.Grid(ctx, *dims)
    return cfg, B, O.BCSR.from_stencil(*dims, B), g


def apply_gpu(rsv, A, n, r, **kw):
    M = rsv.Precond(A, local_solver=rsv.LOCAL_ILUT, **kw)
    z = torch.zeros(n, dtype=torch.float64, device="cuda")
    M.apply(dev(r), z)
    M.close()
    return z.cpu().numpy()


def bar_of(shift, ref, r):
    """1e-12 of the largest entry; on the literal reading (shift 0) the
    factors amplify r (pivot blocks with condition numbers in the thousands)
    and the sweeps' rounding with it, so the bar scales with max|z|/max|r|."""
    amp = np.max(np.abs(ref)) / np.max(np.abs(r))
    return 1e-12 if shift == 2.0 else 1e-12 * max(1.0, amp)


GRIDS = [(20, 20, 10), (13, 9, 5), (1, 1, 7), (7, 1, 1), (17, 3, 19), (9, 16, 33)]
PT = [(-1, 1e-3), (2, 1e-2), (5, 1e-4), (1, 0.0), (8, 1e-3)]


@pytest.mark.parametrize("dims", GRIDS)
@pytest.mark.parametrize("p,tol", PT)
@pytest.mark.parametrize("shift", [2.0, 0.0])
def test_whole_grid_ilut_apply(rsv, ctx, dims, p, tol, shift):
    log("ilut", dims, p, tol, shift)
    cfg, B, Ao, g = sysm(rsv, ctx, dims, 3, shift)
    A = rsv.Matrix(g, dev(B))
    n = 3 * cfg.ncell
    r = I.test_vector(3, n)
    z = apply_gpu(rsv, A, n, r, type=rsv.PC_BILU0, ilut_p=p, ilut_tol=tol)
    ref = O.ILU(Ao, ilut=(p, tol)).apply(r)
    err = np.max(np.abs(z - ref)) / np.max(np.abs(ref))
    bar = bar_of(shift, ref, r)
    log("  error", err, "bar", bar)
    assert err <= bar
    A.close(); g.close()


def test_ilut_apply_large_subdomain(rsv, ctx):
    """The whole 64x64x32 grid as one subdomain: at least 256 rows per level
    on average, so the apply runs one launch per level."""
    dims = (64, 64, 32)
    cfg, B, Ao, g = sysm(rsv, ctx, dims, 13, 2.0)
    A = rsv.Matrix(g, dev(B))
    n = 3 * cfg.ncell
    r = I.test_vector(14, n)
    z = apply_gpu(rsv, A, n, r, type=rsv.PC_BILU0)
    ref = O.ILU(Ao, ilut=(-1, 1e-3)).apply(r)
    err = np.max(np.abs(z - ref)) / np.max(np.abs(ref))
    log("  error", err)
    assert err <= bar_of(2.0, ref, r)
    A.close(); g.close()


def test_ras_ilut_apply_large_subdomains(rsv, ctx):
    """Two RAS subdomains of 49x64x32 cells with ILUT(-1, 1e-3) local
    factors: the size at which the apply takes one launch per level."""
    dims, parts = (96, 64, 32), (2, 1, 1)
    cfg, B, Ao, g = sysm(rsv, ctx, dims, 15, 2.0)
    A = rsv.Matrix(g, dev(B))
    n = 3 * cfg.ncell
    r = I.test_vector(16, n)
    z = apply_gpu(rsv, A, n, r, type=rsv.PC_RAS, ras_px=parts[0], ras_py=parts[1], ras_pz=parts[2],
                  ras_overlap=1, ilut_p=-1, ilut_tol=1e-3)
    ref = O.RAS(Ao, dims, parts, 1, ilut=(-1, 1e-3)).apply(r)
    err = np.max(np.abs(z - ref)) / np.max(np.abs(ref))
    log("  error", err)
    assert err <= bar_of(2.0, ref, r)
    A.close(); g.close()


@pytest.mark.parametrize("dims,parts,ov", [((20, 20, 10), (2, 2, 2), 1), ((13, 9, 5), (3, 2, 1), 1),
                                           ((17, 3, 19), (2, 1, 3), 2), ((9, 16, 33), (1, 2, 4), 0),
                                           ((32, 32, 16), (4, 4, 4), 1)])
@pytest.mark.parametrize("p,tol", [(-1, 1e-3), (4, 1e-4)])
@pytest.mark.parametrize("shift", [2.0, 0.0])
def test_ras_ilut_apply(rsv, ctx, dims, parts, ov, p, tol, shift):
    log("ras ilut", dims, parts, ov, p, tol, shift)
    cfg, B, Ao, g = sysm(rsv, ctx, dims, 5, shift)
    A = rsv.Matrix(g, dev(B))
    n = 3 * cfg.ncell
    r = I.test_vector(6, n)
    z = apply_gpu(rsv, A, n, r, type=rsv.PC_RAS, ras_px=parts[0], ras_py=parts[1], ras_pz=parts[2],
                  ras_overlap=ov, ilut_p=p, ilut_tol=tol)
    ref = O.RAS(Ao, dims, parts, ov, ilut=(p, tol)).apply(r)
    err = np.max(np.abs(z - ref)) / np.max(np.abs(ref))
    bar = bar_of(shift, ref, r)
    log("  error", err, "bar", bar)
    assert err <= bar
    A.close(); g.close()


@pytest.mark.parametrize("case", ["C1-literal", "C2"])
def test_gmres_ras_ilut_against_oracle(rsv, ctx, case):
    if case == "C2":
        cfg = I.preset("C2", seed=0)
        parts = (4, 4, 4)
    else:
        cfg = I.preset("C1", seed=0)
        parts = (2, 2, 2)
    dims = (cfg.nx, cfg.ny, cfg.nz)
    B = I.blocks(cfg)
    Ao = O.BCSR.from_stencil(*dims, B)
    g = rsv.Grid(ctx, *dims)
    A = rsv.Matrix(g, dev(B))
    del B
    xt = I.x_true(cfg)
    bo = Ao.spmv(xt)
    M = rsv.Precond(A, type=rsv.PC_RAS, ras_px=parts[0], ras_py=parts[1], ras_pz=parts[2], ras_overlap=1,
                    local_solver=rsv.LOCAL_ILUT)
    x = torch.zeros(3 * cfg.ncell, dtype=torch.float64, device="cuda")
    st = rsv.solve(A, M, dev(bo), x, method=rsv.GMRES, restart=30, tol=1e-8, maxit=3000, record_history=1)
    xg = x.cpu().numpy()
    rr = np.linalg.norm(bo - Ao.spmv(xg)) / np.linalg.norm(bo)
    ref = O.gmres(Ao, bo, pc=O.RAS(Ao, dims, parts, 1, ilut=(-1, 1e-3)), m=30, tol=1e-8, maxit=3000, hist=True)
    log(f"{case}: its {st['its']} (oracle {ref['its']}), relres {rr:.3e}, x vs oracle {rel(xg, ref['x']):.2e}")
    assert st["status"] == 0 and ref["rc"] == 0 and rr <= 1e-8
    assert rel(xg, ref["x"]) <= 1e-6
    assert abs(st["its"] - ref["its"]) <= max(2, 0.05 * ref["its"])
    k = min(10, len(ref["hist"]), len(st["hist"]))
    assert np.allclose(st["hist"][:k], ref["hist"][:k], rtol=1e-8, atol=0)
    M.close(); A.close(); g.close()


def test_cpr_with_ilut_stage(rsv, ctx):
    dims = (20, 20, 10)
    cfg, B, Ao, g = sysm(rsv, ctx, dims, 9, 0.0)
    A = rsv.Matrix(g, dev(B))
    n = 3 * cfg.ncell
    f = I.test_vector(9, n)
    M = rsv.Precond(A, type=rsv.PC_CPR, cpr_stage=rsv.PC_RAS, ras_px=2, ras_py=2, ras_pz=2, ras_overlap=1,
                    local_solver=rsv.LOCAL_ILUT)
    z = torch.zeros(n, dtype=torch.float64, device="cuda")
    M.apply(dev(f), z)
    ref = OC.CPR(Ao, dims, O.RAS(Ao, dims, (2, 2, 2), 1, ilut=(-1, 1e-3))).apply(f)
    amp = np.max(np.abs(ref)) / np.max(np.abs(f))
    assert np.max(np.abs(z.cpu().numpy() - ref)) <= 1e-12 * max(1.0, amp) * np.max(np.abs(ref))
    M.close(); A.close(); g.close()


def test_ilut_errors(rsv, ctx):
    cfg, B, Ao, g = sysm(rsv, ctx, (8, 6, 4), 10)
    A = rsv.Matrix(g, dev(B))
    for kw in (dict(ilut_p=-2), dict(ilut_p=33), dict(ilut_tol=-1.0), dict(ilut_tol=float("inf")),
               dict(iluk_level=1), dict(precision=rsv.FP32), dict(local_solver=2)):
        args = dict(type=rsv.PC_RAS, ras_px=2, ras_py=2, ras_pz=1, local_solver=rsv.LOCAL_ILUT)
        args.update(kw)
        with pytest.raises(rsv.RsvError) as e:
            rsv.Precond(A, **args)
        assert e.value.status == rsv.ERR_ARG, kw
    # a singular diagonal block that no elimination touches (cell 0, the first row)
    B2 = B.copy()
    B2[0, 3] = 0.0
    A2 = rsv.Matrix(g, dev(B2))
    with pytest.raises(rsv.RsvError) as e:
        rsv.Precond(A2, type=rsv.PC_BILU0, local_solver=rsv.LOCAL_ILUT, ilut_tol=1e300)
    assert e.value.status == rsv.ERR_ZERO_PIVOT and e.value.bad_cell == 0
    A2.close()
    # no dropping: the fill of a 40x40 band outgrows the work row
    A.close(); g.close()
    cfg, B, Ao, g = sysm(rsv, ctx, (40, 40, 6), 11)
    A = rsv.Matrix(g, dev(B))
    with pytest.raises(rsv.RsvError) as e:
        rsv.Precond(A, type=rsv.PC_BILU0, local_solver=rsv.LOCAL_ILUT, ilut_p=32, ilut_tol=0.0)
    assert e.value.status == rsv.ERR_ARG
    A.close(); g.close()
    # a band too wide for LDS
    cfg, B, Ao, g = sysm(rsv, ctx, (256, 256, 2), 12)
    A = rsv.Matrix(g, dev(B))
    with pytest.raises(rsv.RsvError) as e:
        rsv.Precond(A, type=rsv.PC_BILU0, local_solver=rsv.LOCAL_ILUT)
    assert e.value.status == rsv.ERR_ARG
    A.close(); g.close()
