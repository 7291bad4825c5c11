"""Pins for the oracle's Hilbert space-filling-curve partition (Space-filling
Partitioning Method section): the defining properties of a Hilbert curve on
the lattice of cell centres (a bijection onto the keys, consecutive points
face neighbours, start and end corners, nested levels), the paper's coordinate
scaling, the equal-count cut of the curve against numpy's stable sort, and
the partition-quality measures (Partition Quality subsection) against brute
force and the closed forms of a partition into octants.  No GPU needed."""
import itertools

import numpy as np
import pytest

from oracle import hsfc as H


def lattice(m):
    n = 2 ** m
    pts = np.array(list(itertools.product(range(n), repeat=3)))
    return pts, (pts + 0.5) / n


@pytest.mark.parametrize("m", [1, 2, 3, 4])
def test_keys_are_a_bijection_and_consecutive_points_are_neighbours(m):
    pts, c = lattice(m)
    keys = np.array([H.key3(p, m) for p in c], dtype=np.uint64)
    assert np.array_equal(np.sort(keys), np.arange(8 ** m, dtype=np.uint64))
    order = pts[np.argsort(keys)]
    steps = np.abs(np.diff(order, axis=0)).sum(axis=1)
    assert np.all(steps == 1)                      # each step moves to a face neighbour
    assert tuple(order[0]) == (0, 0, 0) and tuple(order[-1]) == (0, 0, 2 ** m - 1)


def test_level_one_order_and_nesting():
    # the first level visits the octants in a Gray-code order (one bit per step),
    # x carrying weight 4, y 2 and z 1 in the octant index
    _, c = lattice(1)
    order = sorted(range(8), key=lambda q: H.key3(c[q], 1))
    octs = [tuple(lattice(1)[0][q]) for q in order]
    assert octs == [(0, 0, 0), (1, 0, 0), (1, 1, 0), (0, 1, 0), (0, 1, 1), (1, 1, 1), (1, 0, 1), (0, 0, 1)]
    # a level-(m+1) key extends the level-m key of the parent cell by one digit
    pts, c = lattice(3)
    for p, cc in zip(pts[::7], c[::7]):
        parent = (p // 2 + 0.5) / 4
        assert H.key3(cc, 3) >> 3 == H.key3(parent, 2)
    # levels are read from the most significant coordinate bit down
    assert H.key3([0.5 + 1e-9, 0.25, 0.25], 1) == H.key3([0.9, 0.1, 0.4], 1)


def test_paper_coordinate_scaling_and_range():
    # [0,1] is scaled by 2^32 - 1 and truncated: 1.0 lands in the last cell of every level
    for m in (1, 5, 21):
        assert H.key3([1.0, 1.0, 1.0], m) == H.key3([1 - 2.0 ** -40] * 3, m)
        assert H.key3([0.0, 0.0, 0.0], m) == 0
    assert H.key3([0.3, 0.6, 0.9], 21) < 8 ** 21
    for bad in ([-0.1, 0.5, 0.5], [0.5, 1.5, 0.5], [np.nan, 0.5, 0.5]):
        with pytest.raises(ValueError):
            H.key3(bad, 5)
    with pytest.raises(ValueError):
        H.key3([0.5] * 3, 22)


@pytest.mark.parametrize("dims", [(5, 4, 3), (16, 16, 16), (13, 9, 7), (1, 1, 9)])
def test_grid_keys_scale_by_the_largest_extent(dims):
    nx, ny, nz = dims
    L = max(dims)
    keys = H.grid_keys(dims, 10)
    i, j, k = np.meshgrid(np.arange(nx), np.arange(ny), np.arange(nz), indexing="ij")
    for q in range(0, nx * ny * nz, max(1, nx * ny * nz // 50)):
        ii, jj, kk = q % nx, (q // nx) % ny, q // (nx * ny)
        assert keys[q] == H.key3([(ii + 0.5) / L, (jj + 0.5) / L, (kk + 0.5) / L], 10)


@pytest.mark.parametrize("dims,levels,nparts", [((16, 16, 16), 4, 8), ((13, 9, 7), 6, 5), ((20, 20, 10), 5, 64),
                                                ((6, 5, 4), 2, 7), ((3, 3, 3), 1, 4)])
def test_partition_is_the_equal_count_cut_of_the_curve(dims, levels, nparts):
    keys = H.grid_keys(dims, levels)         # level 1-2 on the small grids: many equal keys
    part = H.partition(keys, nparts)
    n = len(keys)
    ranks = np.empty(n, np.int64)
    ranks[np.argsort(keys, kind="stable")] = np.arange(n)
    assert np.array_equal(part, (ranks * nparts) // n)
    sizes = np.bincount(part, minlength=nparts)
    assert sizes.max() - sizes.min() <= 1
    for p in range(nparts - 1):
        assert keys[part == p].max() <= keys[part == p + 1].min()


def brute_quality(dims, part, nparts):
    nx, ny, nz = dims
    P = part.reshape(nz, ny, nx)
    size = np.bincount(part, minlength=nparts)
    f = np.zeros(nparts, np.int64)
    b = np.zeros(nparts, np.int64)
    nb = [set() for _ in range(nparts)]
    # every face of the grid once: boundary faces belong to their cell, inner faces to both sides' parts
    for axis in range(3):
        lo = np.take(P, [0], axis=2 - axis).ravel()
        hi = np.take(P, [P.shape[2 - axis] - 1], axis=2 - axis).ravel()
        np.add.at(f, lo, 1)
        np.add.at(f, hi, 1)
        a = np.take(P, range(P.shape[2 - axis] - 1), axis=2 - axis).ravel()
        c = np.take(P, range(1, P.shape[2 - axis]), axis=2 - axis).ravel()
        same = a == c
        np.add.at(f, a[same], 1)
        np.add.at(f, a[~same], 1)
        np.add.at(f, c[~same], 1)
        np.add.at(b, a[~same], 1)
        np.add.at(b, c[~same], 1)
        for x, y in zip(a[~same], c[~same]):
            nb[x].add(y)
            nb[y].add(x)
    conn = np.array([len(s) for s in nb])
    r = b / f
    return [nparts * size.max() / size.sum(), r.max(), b.sum() / (f.sum() - b.sum()), r.mean(), conn.max()], \
        np.stack([size, f, b, conn], axis=1)


@pytest.mark.parametrize("dims,nparts", [((6, 5, 4), 7), ((13, 9, 7), 5), ((8, 8, 8), 64), ((10, 1, 1), 3)])
def test_quality_against_brute_force(dims, nparts):
    part = H.partition(H.grid_keys(dims, 8), nparts)
    q, per = H.quality(dims, part, nparts)
    qb, perb = brute_quality(dims, part, nparts)
    assert np.array_equal(per, perb)
    assert np.allclose(q, qb, rtol=1e-15, atol=0)


@pytest.mark.parametrize("m", [2, 3, 4])
def test_octant_partition_closed_forms(m):
    """On a 2^m cube the Hilbert cut into 8 parts is the 8 octants (the curve
    fills one octant before the next): each is a cube of side s = 2^(m-1)
    with s^3 cells, 3 s^2 (s + 1) faces of which 3 s^2 face other octants,
    and 3 face-neighbour octants; so f_p = 1, r_M = mean = 1/(s+1),
    r_G = 24 s^2 / (24 s^2 (s+1) - 24 s^2) = 1/s, c = 3."""
    n = 2 ** m
    s = n // 2
    dims = (n, n, n)
    part = H.partition(H.grid_keys(dims, m), 8)
    P = part.reshape(n, n, n)
    for z in (0, 1):
        for y in (0, 1):
            for x in (0, 1):
                assert len(np.unique(P[z * s:(z + 1) * s, y * s:(y + 1) * s, x * s:(x + 1) * s])) == 1
    q, per = H.quality(dims, part, 8)
    assert np.all(per[:, 0] == s ** 3) and np.all(per[:, 1] == 3 * s * s * (s + 1))
    assert np.all(per[:, 2] == 3 * s * s) and np.all(per[:, 3] == 3)
    assert q[0] == 1.0 and q[4] == 3.0
    assert q[1] == pytest.approx(1 / (s + 1), rel=1e-15) and q[3] == pytest.approx(1 / (s + 1), rel=1e-15)
    assert q[2] == pytest.approx(1 / s, rel=1e-15)
