"""Pins for the oracle's ILU(k) (level-of-fill incomplete LU, the RAS local
solver ILUK of the RAS parameter figure): the level-1 pattern of the 7-point
stencil in closed form, nested patterns ending in the exact LU, the ILU
characterisation (LU)_ij = A_ij on the pattern, a dense solve of the formed
factors, ILU(0) as the level-0 case, and RAS with ILU(k) local solvers by its
special cases.  No GPU needed."""
import itertools

import numpy as np
import pytest

from paper_1602_05901_amd import inputs as I
import oracle as O

OFF = [(0, 0, -1), (0, -1, 0), (-1, 0, 0), (0, 0, 0), (1, 0, 0), (0, 1, 0), (0, 0, 1)]


def small(dims, seed=0, shift=0.0, sigma=1.0):
    cfg = I.GenConfig(*dims, I.LNK_IID, sigma, 0.0, shift, 0, 1e3, 1.0, seed)
    B = I.blocks(cfg)
    return cfg, B, O.BCSR.from_stencil(*dims, B)


def dense(A):
    return O.bcsr_to_dense(*A.export())


def factors(F, n):
    rp, col, val = F.factors()
    L, U = np.eye(3 * n), np.zeros((3 * n, 3 * n))
    for i in range(n):
        for p in range(rp[i], rp[i + 1]):
            j = col[p]
            (L if j < i else U)[3 * i:3 * i + 3, 3 * j:3 * j + 3] = val[p]
    return L, U, rp, col


@pytest.mark.parametrize("dims", [(4, 3, 3), (5, 4, 2), (3, 3, 3), (6, 1, 4)])
def test_level_one_pattern_of_the_seven_point_stencil(dims):
    """Level-1 fill of the 7-point stencil in natural order: eliminating the
    -a neighbour brings in its +b neighbour, so every cell gains c - e_a + e_b
    (a != b) wherever that cell exists, at level 1, and nothing else."""
    nx, ny, nz = dims
    cfg, B, A = small(dims)
    rp, col, lev = O.iluk_pattern(A, 1)
    E = [(1, 0, 0), (0, 1, 0), (0, 0, 1)]
    for c in range(cfg.ncell):
        i, j, k = c % nx, (c // nx) % ny, c // (nx * ny)
        want = {}
        for d in OFF:
            ii, jj, kk = i + d[0], j + d[1], k + d[2]
            if 0 <= ii < nx and 0 <= jj < ny and 0 <= kk < nz:
                want[ii + nx * (jj + ny * kk)] = 0
        for a, b in itertools.permutations(range(3), 2):
            ii, jj, kk = i - E[a][0] + E[b][0], j - E[a][1] + E[b][1], k - E[a][2] + E[b][2]
            if 0 <= ii < nx and 0 <= jj < ny and 0 <= kk < nz:
                want.setdefault(ii + nx * (jj + ny * kk), 1)
        got = dict(zip(col[rp[c]:rp[c + 1]].tolist(), lev[rp[c]:rp[c + 1]].tolist()))
        assert got == want, c
        assert list(col[rp[c]:rp[c + 1]]) == sorted(got)


def test_patterns_nest_and_end_in_the_exact_lu():
    dims = (3, 3, 2)
    cfg, B, A = small(dims, 1, 2.0)
    n = cfg.ncell
    prev = None
    for k in range(0, 6):
        rp, col, lev = O.iluk_pattern(A, k)
        pat = {(i, j) for i in range(n) for j in col[rp[i]:rp[i + 1]]}
        assert lev.max() <= k
        if prev is not None:
            assert prev <= pat
        prev = pat
    # a level beyond any path length keeps every fill position: the exact LU
    F = O.ILU(A, level=3 * n)
    L, U, _, _ = factors(F, n)
    D = dense(A)
    assert np.allclose(L @ U, D, rtol=0, atol=1e-12 * np.abs(D).max())
    b = A.spmv(I.x_true(cfg))
    out = O.gmres(A, b, pc=F, m=30, tol=1e-12, maxit=5)
    assert out["rc"] == O.OK and out["its"] == 1


@pytest.mark.parametrize("k", [1, 2, 3])
@pytest.mark.parametrize("dims,shift", [((4, 3, 3), 0.0), ((5, 4, 2), 2.0)])
def test_iluk_characterisation_and_apply(dims, shift, k):
    cfg, B, A = small(dims, 2, shift)
    n = cfg.ncell
    D = dense(A)
    F = O.ILU(A, level=k)
    L, U, rp, col = factors(F, n)
    LU = L @ U
    for i in range(n):
        for j in col[rp[i]:rp[i + 1]]:
            blk = (slice(3 * i, 3 * i + 3), slice(3 * j, 3 * j + 3))
            assert np.max(np.abs(LU[blk] - D[blk])) <= 1e-12 * np.abs(D).max()
    r = I.test_vector(3, 3 * n)
    assert np.allclose(F.apply(r), np.linalg.solve(LU, r), rtol=1e-11, atol=1e-13)
    # more levels: a closer factorisation of A
    L0, U0, _, _ = factors(O.ILU(A, level=k - 1), n)
    assert np.linalg.norm(LU - D) < np.linalg.norm(L0 @ U0 - D)


def test_level_zero_is_ilu0():
    cfg, B, A = small((5, 4, 3), 4)
    r = I.test_vector(5, 3 * cfg.ncell)
    assert np.array_equal(O.ILU(A, level=0).apply(r), O.ILU(A).apply(r))


@pytest.mark.parametrize("k", [1, 2])
def test_ras_with_iluk_local_solvers(k):
    dims = (8, 6, 4)
    cfg, B, A = small(dims, 6, 2.0)
    r = I.test_vector(7, 3 * cfg.ncell)
    ilu = O.ILU(A, level=k).apply(r)
    assert np.allclose(O.RAS(A, dims, (1, 1, 1), 1, level=k).apply(r), ilu, rtol=1e-13, atol=1e-15)
    assert np.allclose(O.RAS(A, dims, (2, 2, 2), sum(dims), level=k).apply(r), ilu, rtol=1e-12, atol=1e-14)
    # overlap 0: every box factored on its own, ILU(k) of the block-diagonal part
    R0 = O.RAS(A, dims, (2, 3, 1), 0, level=k)
    own = O.RAS(A, dims, (2, 3, 1), 0).owner()
    nx, ny, nz = dims
    B0 = B.copy()
    for c in range(cfg.ncell):
        i, j, kk = c % nx, (c // nx) % ny, c // (nx * ny)
        for s, (di, dj, dk) in enumerate(OFF):
            ii, jj, k2 = i + di, j + dj, kk + dk
            if s != 3 and 0 <= ii < nx and 0 <= jj < ny and 0 <= k2 < nz and own[ii + nx * (jj + ny * k2)] != own[c]:
                B0[c, s] = 0.0
    A0 = O.BCSR.from_stencil(*dims, B0)
    assert np.allclose(R0.apply(r), O.ILU(A0, level=k).apply(r), rtol=1e-12, atol=1e-14)


def test_iluk_reduces_gmres_steps_on_c1():
    cfg = I.preset("C1", seed=3, m_shift=2.0)
    A = O.BCSR.from_stencil(cfg.nx, cfg.ny, cfg.nz, I.blocks(cfg))
    b = A.spmv(I.x_true(cfg))
    its = [O.gmres(A, b, pc=O.ILU(A, level=k), m=30, tol=1e-8, maxit=500)["its"] for k in (0, 1, 2)]
    assert its[2] <= its[1] <= its[0]
