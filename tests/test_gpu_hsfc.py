"""GPU parity of the Hilbert space-filling-curve keys, the equal-count curve
partition and the partition-quality measures (Space-filling Partitioning
Method section) against the oracle, through the C ABI.  Integer results are
bit-exact (keys, part numbers, per-part face counts); the ratios of the
quality measures to FP64 rounding of their sums.  Sizes span one tile of the
radix sort up to the 512x512x128 grid, with heavy key ties (few levels) and
the longest keys (21 levels, 8 sort passes)."""
import sys

import numpy as np
import pytest

torch = pytest.importorskip("torch")

from paper_1602_05901_amd import inputs as I  # noqa: E402
from oracle import hsfc as H  # noqa: E402

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


def check_q(q, qo, nparts):
    """Load imbalance, max b/f, the global index and max connectivity come from
    the same integers by the same single operations: equal.  The average
    sums nparts ratios in another order: within nparts rounding errors."""
    assert q[0] == qo[0] and q[1] == qo[1] and q[2] == qo[2] and q[4] == qo[4]
    assert abs(q[3] - qo[3]) <= nparts * 2.3e-16 * qo[3]


def points(n, seed):
    p = I.uniform(seed, 7, 3 * n, 0.0, 1.0).reshape(n, 3)
    p[:8] = [[0, 0, 0], [1, 1, 1], [1, 0, 0], [0, 1, 0], [0, 0, 1], [0.5, 0.5, 0.5], [0.25, 0.75, 1.0],
             [np.nextafter(0.5, 0), 0.5, np.nextafter(1.0, 0)]]
    return p


@pytest.mark.parametrize("levels", [1, 2, 5, 10, 21])
def test_point_keys_bit_exact(rsv, ctx, levels):
    p = points(20000, levels)
    keys = torch.zeros(len(p), dtype=torch.int64, device="cuda")
    rsv.hsfc_keys(ctx, dev(p), levels, keys)
    got = keys.cpu().numpy().view(np.uint64)
    ref = np.array([H.key3(q, levels) for q in p], dtype=np.uint64)
    assert np.array_equal(got, ref)


def test_point_keys_reject_out_of_range(rsv, ctx):
    for bad in ([0.5, -0.25, 0.5], [0.5, 0.5, 1.0 + 1e-12], [np.nan, 0.5, 0.5]):
        p = points(300, 3)
        p[123] = bad
        keys = torch.zeros(len(p), dtype=torch.int64, device="cuda")
        with pytest.raises(rsv.RsvError) as e:
            rsv.hsfc_keys(ctx, dev(p), 8, keys)
        assert e.value.status == rsv.ERR_ARG
    with pytest.raises(rsv.RsvError):
        rsv.hsfc_keys(ctx, dev(points(10, 1)), 22, torch.zeros(10, dtype=torch.int64, device="cuda"))


GRIDS = [((8, 8, 8), 3, 8), ((13, 9, 7), 6, 5), ((20, 20, 10), 2, 64), ((1, 1, 9), 4, 3), ((64, 64, 32), 7, 64),
         ((130, 70, 9), 8, 100), ((5, 4, 3), 1, 7), ((3, 2, 2), 21, 20)]


@pytest.mark.parametrize("dims,levels,nparts", GRIDS)
def test_grid_partition_and_quality_bit_exact(rsv, ctx, dims, levels, nparts):
    log("hsfc", dims, levels, nparts)
    g = rsv.Grid(ctx, *dims)
    n = g.ncell
    keys = torch.zeros(n, dtype=torch.int64, device="cuda")
    g.hsfc_keys(levels, keys)
    kref = H.grid_keys(dims, levels)
    assert np.array_equal(keys.cpu().numpy().view(np.uint64), kref)
    part = torch.full((n,), -1, dtype=torch.int32, device="cuda")
    rsv.hsfc_partition(ctx, keys, levels, nparts, part)
    pref = H.partition(kref, nparts)
    assert np.array_equal(part.cpu().numpy(), pref)
    q, per = g.partition_quality(part, nparts)
    qo, pero = H.quality(dims, pref, nparts)
    assert np.array_equal(per, pero)
    check_q(q, qo, nparts)
    g.close()


def test_partition_of_many_random_keys_21_levels(rsv, ctx):
    """The longest keys (63 bits, eight sort passes) over 3 M random points:
    many tiles, a ragged last tile, and ties only where points coincide."""
    n = 3_000_017
    p = points(n, 99)
    p[1000:1100] = p[5]            # a run of equal points (equal keys, ordered by index)
    keys = torch.zeros(n, dtype=torch.int64, device="cuda")
    rsv.hsfc_keys(ctx, dev(p), 21, keys)
    part = torch.zeros(n, dtype=torch.int32, device="cuda")
    rsv.hsfc_partition(ctx, keys, 21, 4096, part)
    kh = keys.cpu().numpy().view(np.uint64)
    assert np.array_equal(part.cpu().numpy(), H.partition(kh, 4096))


def test_top_down_numbering_permutes_the_rows(rsv, ctx):
    dims = (12, 10, 6)
    nx, ny, nz = dims
    g = rsv.Grid(ctx, *dims, rsv.TOP_DOWN)
    keys = torch.zeros(g.ncell, dtype=torch.int64, device="cuda")
    g.hsfc_keys(9, keys)
    ref = H.grid_keys(dims, 9)
    c = np.arange(g.ncell)
    perm = ((nz - 1 - c // (nx * ny)) * ny + (c // nx) % ny) * nx + c % nx   # row of natural cell c
    assert np.array_equal(keys.cpu().numpy().view(np.uint64)[perm], ref)
    g.close()


def test_quality_rejects_bad_part_numbers(rsv, ctx):
    g = rsv.Grid(ctx, 6, 5, 4)
    part = torch.zeros(g.ncell, dtype=torch.int32, device="cuda")
    part[17] = 9
    with pytest.raises(rsv.RsvError) as e:
        g.partition_quality(part, 8)
    assert e.value.status == rsv.ERR_ARG
    g.close()


@pytest.mark.parametrize("nparts", [64, 4096])
def test_C5_grid_partition_full_size(rsv, ctx, nparts):
    """The 512x512x128 grid (33.5 M cells), in the configuration the bench
    times: keys at 9 levels, the partition and its quality, all against the
    oracle in full."""
    dims = (512, 512, 128)
    log("hsfc C5", nparts)
    g = rsv.Grid(ctx, *dims)
    n = g.ncell
    keys = torch.zeros(n, dtype=torch.int64, device="cuda")
    g.hsfc_keys(9, keys)
    kref = H.grid_keys(dims, 9)
    assert np.array_equal(keys.cpu().numpy().view(np.uint64), kref)
    part = torch.zeros(n, dtype=torch.int32, device="cuda")
    rsv.hsfc_partition(ctx, keys, 9, nparts, part)
    pref = H.partition(kref, nparts)
    assert np.array_equal(part.cpu().numpy(), pref)
    q, per = g.partition_quality(part, nparts)
    qo, pero = H.quality(dims, pref, nparts)
    log("  quality", q)
    assert np.array_equal(per, pero)
    check_q(q, qo, nparts)
    g.close()
