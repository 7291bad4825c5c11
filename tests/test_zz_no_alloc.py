"""The entry point that allocates nothing (rsv_spmv_noalloc), through the C
ABI: its product equals rsv_spmv's bit for bit (the same kernels on the same
inputs) and the oracle's to the SpMV bar, on two calls in a row -- the
second on a smaller grid -- and it never reserves the matrix's workspace.
A grid too large for the fixed scratch is refused before anything runs."""
import sys

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


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def test_spmv_noalloc_equals_spmv_twice(rsv):
    ctx = rsv.Context(0)
    for dims, seed in (((128, 128, 64), 3), ((13, 9, 5), 4)):      # the second call on a smaller grid
        log("spmv_noalloc", dims)
        cfg = I.GenConfig(*dims, I.LNK_IID, 2.0, 0.0, 2.0, 0, 1e3, 1.0, seed)
        B = I.blocks(cfg)
        g = rsv.Grid(ctx, *dims)
        A = rsv.Matrix(g, dev(B))
        before = A.device_bytes
        n = 3 * cfg.ncell
        x = I.test_vector(seed, n)
        y0 = I.test_vector(seed + 1, n)
        y_na = dev(y0)
        A.spmv_noalloc(dev(x), y_na, alpha=0.5, beta=-2.0)
        assert A.device_bytes == before          # no workspace was reserved
        y_ws = dev(y0)
        A.spmv(dev(x), y_ws, alpha=0.5, beta=-2.0)
        assert torch.equal(y_na, y_ws)
        Ao = O.BCSR.from_stencil(*dims, B)
        ref = 0.5 * Ao.spmv(x) - 2.0 * y0
        scale = 0.5 * O.BCSR.from_stencil(*dims, np.abs(B)).spmv(np.abs(x)) + 2.0 * np.abs(y0)
        assert np.all(np.abs(y_na.cpu().numpy() - ref) <= 1e-12 * scale)
        A.close(); g.close()
    ctx.close()


def test_spmv_noalloc_refuses_a_grid_beyond_the_scratch(rsv):
    ctx = rsv.Context(0)
    g = rsv.Grid(ctx, 128, 128, 128)           # 2 x 3 x 2^21 slots x 8 bytes = 96 MiB > 64 MiB
    cfg = I.GenConfig(128, 128, 128, I.LNK_IID, 1.0, 0.0, 2.0, 0, 1e3, 1.0, 5)
    A = rsv.Matrix(g, dev(I.blocks(cfg)))
    n = 3 * cfg.ncell
    x = torch.zeros(n, dtype=torch.float64, device="cuda")
    y = torch.full((n,), 7.0, dtype=torch.float64, device="cuda")
    with pytest.raises(rsv.RsvError) as e:
        A.spmv_noalloc(x, y)
    assert e.value.status == rsv.ERR_ARG
    assert float(y.min()) == 7.0 and float(y.max()) == 7.0     # nothing ran
    A.close(); g.close(); ctx.close()
