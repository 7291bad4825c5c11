"""Pins for the oracle's scalar path (the paper's Poisson Equation example:
GMRES(30) with RAS, overlap one, ILU(0) local solves): the product against a
dense matrix built straight from the coefficients and the Laplacian's row
sums; ILU(0) by its characterisation, the exact LU of a 1-D grid and a dense
solve; RAS by its special cases; GMRES by the dense least-squares minimiser
and by the closed-form spectrum of the 7-point Laplacian.  No GPU needed."""
import itertools

import numpy as np
import pytest

from paper_1602_05901_amd import inputs as I
from oracle import scalar as S
import oracle as O

OFF = [(0, 0, -1), (0, -1, 0), (-1, 0, 0), (0, 0, 0), (1, 0, 0), (0, 1, 0), (0, 0, 1)]


def coef(dims, sigma=0.0, seed=0):
    cfg = I.GenConfig(*dims, I.LNK_IID, sigma, 0.0, 0.0, 0, 1e3, 1.0, seed)
    return cfg, I.poisson(cfg, I.lnk(cfg) if sigma > 0 else None)


def dense_of(dims, C):
    nx, ny, nz = dims
    n = nx * ny * nz
    D = np.zeros((n, n))
    for k, j, i in itertools.product(range(nz), range(ny), range(nx)):
        c = i + nx * (j + ny * k)
        for s, (di, dj, dk) in enumerate(OFF):
            ii, jj, kk = i + di, j + dj, k + dk
            if 0 <= ii < nx and 0 <= jj < ny and 0 <= kk < nz:
                D[c, ii + nx * (jj + ny * kk)] = C[c, s]
    return D


@pytest.mark.parametrize("dims,sigma", [((4, 3, 2), 0.0), ((5, 1, 1), 1.0), ((3, 3, 3), 2.0), ((1, 1, 1), 0.0)])
def test_spmv_against_dense(dims, sigma):
    cfg, C = coef(dims, sigma, 1)
    A = S.CSR(*dims, C)
    x = I.test_vector(3, cfg.ncell)
    D = dense_of(dims, C)
    assert np.allclose(A.spmv(x), D @ x, rtol=1e-14, atol=1e-14)
    assert np.array_equal(A.dense(), D)


def test_laplacian_row_sums_count_boundary_faces():
    dims = (6, 5, 4)
    nx, ny, nz = dims
    cfg, C = coef(dims)
    A = S.CSR(*dims, C)
    rs = A.spmv(np.ones(cfg.ncell))
    i, j, k = np.meshgrid(np.arange(nx), np.arange(ny), np.arange(nz), indexing="ij")
    faces = sum((a == v).astype(float) for a, v in ((i, 0), (i, nx - 1), (j, 0), (j, ny - 1), (k, 0), (k, nz - 1)))
    assert np.array_equal(rs, faces.transpose(2, 1, 0).ravel())


def test_pattern_and_nan_errors():
    cfg, C = coef((3, 2, 2))
    bad = C.copy()
    bad[0, 2] = -1.0          # -x neighbour of cell 0 does not exist
    with pytest.raises(O.OracleError):
        S.CSR(3, 2, 2, bad)
    bad = C.copy()
    bad[4, 3] = np.nan
    with pytest.raises(O.OracleError):
        S.CSR(3, 2, 2, bad)


def factors(F, n):
    rp, col, val = F.factors()
    L, U = np.eye(n), np.zeros((n, n))
    for i in range(n):
        for p in range(rp[i], rp[i + 1]):
            (L if col[p] < i else U)[i, col[p]] = val[p]
    return L, U


@pytest.mark.parametrize("dims,sigma", [((4, 3, 3), 0.0), ((5, 4, 2), 1.5)])
def test_ilu0_characterisation_and_apply(dims, sigma):
    cfg, C = coef(dims, sigma, 2)
    A = S.CSR(*dims, C)
    D = A.dense()
    F = S.ILU(A)
    L, U = factors(F, cfg.ncell)
    LU = L @ U
    pat = D != 0
    assert np.max(np.abs(LU[pat] - D[pat])) <= 1e-13 * np.abs(D).max()
    assert np.any(np.abs(LU[~pat]) > 1e-3)        # ILU(0) drops fill on a 3-D grid
    r = I.test_vector(4, cfg.ncell)
    assert np.allclose(F.apply(r), np.linalg.solve(LU, r), rtol=1e-12, atol=1e-14)


def test_ilu0_is_exact_lu_on_a_line():
    cfg, C = coef((9, 1, 1), 2.0, 3)
    A = S.CSR(9, 1, 1, C)
    L, U = factors(S.ILU(A), 9)
    assert np.allclose(L @ U, A.dense(), rtol=0, atol=1e-13)
    b = A.spmv(I.x_true_scalar(cfg))
    out = S.gmres(A, b, pc=S.ILU(A), tol=1e-12, maxit=10)
    assert out["rc"] == O.OK and out["its"] == 1


def test_ilu0_zero_pivot():
    cfg, C = coef((3, 2, 2))
    C = C.copy()
    C[0, 3] = 0.0
    with pytest.raises(O.OracleError) as e:
        S.ILU(S.CSR(3, 2, 2, C))
    assert e.value.rc == O.ERR_ZERO_PIVOT


@pytest.mark.parametrize("dims,sigma", [((8, 6, 4), 0.0), ((7, 5, 5), 1.0)])
def test_ras_special_cases(dims, sigma):
    cfg, C = coef(dims, sigma, 5)
    A = S.CSR(*dims, C)
    D = A.dense()
    r = I.test_vector(6, cfg.ncell)
    ilu = S.ILU(A).apply(r)
    # one subdomain, and an overlap reaching the whole grid, are ILU(0)
    assert np.allclose(S.RAS(A, dims, (1, 1, 1), 1).apply(r), ilu, rtol=1e-14, atol=1e-15)
    assert np.allclose(S.RAS(A, dims, (2, 2, 2), sum(dims)).apply(r), ilu, rtol=1e-13, atol=1e-15)
    # overlap 0: ILU(0) of A with the couplings between boxes removed
    R0 = S.RAS(A, dims, (2, 3, 1), 0)
    owner = np.empty(cfg.ncell, int)
    for s in range(R0.nsub):
        owner[R0.sub_cells(s)] = s
    C0 = C.copy()
    nx, ny, nz = dims
    for c in range(cfg.ncell):
        i, j, k = c % nx, (c // nx) % ny, c // (nx * ny)
        for s, (di, dj, dk) in enumerate(OFF):
            ii, jj, kk = i + di, j + dj, k + dk
            if s != 3 and 0 <= ii < nx and 0 <= jj < ny and 0 <= kk < nz and owner[ii + nx * (jj + ny * kk)] != owner[c]:
                C0[c, s] = 0.0
    assert np.allclose(R0.apply(r), S.ILU(S.CSR(*dims, C0)).apply(r), rtol=1e-14, atol=1e-15)
    # singleton boxes without overlap: Jacobi
    RJ = S.RAS(A, dims, dims, 0)
    assert np.allclose(RJ.apply(r), r / np.diag(D), rtol=1e-15, atol=0)


def test_ras_overlap_is_graph_distance():
    dims = (9, 8, 6)
    cfg, C = coef(dims)
    A = S.CSR(*dims, C)
    R = S.RAS(A, dims, (3, 2, 2), 1)
    nx, ny, nz = dims
    # box (1, 0, 1): x 3..5, y 0..3, z 3..5 plus face neighbours, no edges or corners
    cells = set(R.sub_cells(1 + 3 * (0 + 2 * 1)).tolist())
    core = {i + nx * (j + ny * k) for i in range(3, 6) for j in range(0, 4) for k in range(3, 6)}
    assert core <= cells
    extra = cells - core
    for c in extra:
        i, j, k = c % nx, (c // nx) % ny, c // (nx * ny)
        d = max(0, 3 - i) + max(0, i - 5) + max(0, -j) + max(0, j - 3) + max(0, 3 - k) + max(0, k - 5)
        assert d == 1
    assert len(extra) == 2 * 4 * 3 + 1 * 3 * 3 + 1 * 3 * 4    # both x faces, +y face, -z face (z = 5 is the top)


def test_gmres_first_iterates_minimise_the_residual():
    dims = (4, 3, 3)
    cfg, C = coef(dims, 1.0, 7)
    A = S.CSR(*dims, C)
    D = A.dense()
    F = S.ILU(A)
    L, U = factors(F, cfg.ncell)
    Minv = np.linalg.inv(L @ U)
    b = I.test_vector(8, cfg.ncell)
    for j in (1, 2, 3, 5):
        out = S.gmres(A, b, pc=F, m=30, tol=0.0, maxit=j)
        K = [b]
        for _ in range(j - 1):
            K.append(D @ (Minv @ K[-1]))
        Q, _ = np.linalg.qr(np.array(K).T)
        y, *_ = np.linalg.lstsq(D @ Minv @ Q, b, rcond=None)
        xs = Minv @ (Q @ y)
        assert np.linalg.norm(out["x"] - xs) <= 1e-9 * np.linalg.norm(xs)


def test_full_gmres_steps_bounded_by_distinct_laplacian_eigenvalues():
    """The 7-point Dirichlet Laplacian on n1 x n2 x n3 has the eigenvalues
    sum_d (2 - 2 cos(pi k_d / (n_d + 1))), k_d = 1..n_d; unpreconditioned
    full GMRES ends in at most as many steps as there are distinct values."""
    for dims in ((4, 4, 4), (5, 3, 2)):
        cfg, C = coef(dims)
        A = S.CSR(*dims, C)
        lam = [sum(2 - 2 * np.cos(np.pi * k / (n + 1)) for k, n in zip(ks, dims))
               for ks in itertools.product(*(range(1, n + 1) for n in dims))]
        distinct = len(np.unique(np.round(lam, 9)))
        assert np.allclose(np.sort(np.linalg.eigvalsh(A.dense())), np.sort(lam), atol=1e-12)
        b = I.test_vector(9, cfg.ncell)
        out = S.gmres(A, b, pc=None, m=60, tol=1e-10, maxit=200)
        assert out["rc"] == O.OK and out["its"] <= distinct + 1, (out["its"], distinct)


def test_manufactured_poisson_solves():
    dims = (16, 12, 10)
    cfg, C = coef(dims)
    A = S.CSR(*dims, C)
    xt = I.x_true_scalar(cfg)
    b = A.spmv(xt)
    for pc in (S.ILU(A), S.RAS(A, dims, (2, 2, 2), 1), None):
        out = S.gmres(A, b, pc=pc, m=30, tol=1e-10, maxit=3000)
        assert out["rc"] == O.OK and out["relres"] <= 1e-10
        assert np.linalg.norm(out["x"] - xt) / np.linalg.norm(xt) <= 1e-7
    out = S.bicgstab(A, b, pc=S.RAS(A, dims, (2, 2, 2), 1), tol=1e-10, maxit=3000)
    assert out["rc"] == O.OK and out["relres"] <= 1e-10


def test_ras_on_a_line_is_the_restricted_sum_of_exact_local_solves():
    """On an n x 1 x 1 grid each local matrix is tridiagonal, so its ILU(0)
    is exact: RAS r = sum_s Rtilde_s^T A_s^{-1} R_s r, with Omega_s the box
    plus one cell on each side and only the owned cells written back."""
    n, p = 17, 3
    cfg, C = coef((n, 1, 1), 1.0, 11)
    A = S.CSR(n, 1, 1, C)
    D = A.dense()
    r = I.test_vector(12, n)
    starts = [b * (n // p) + min(b, n % p) for b in range(p + 1)]
    z = np.zeros(n)
    for b in range(p):
        lo, hi = max(0, starts[b] - 1), min(n, starts[b + 1] + 1)
        om = np.arange(lo, hi)
        zl = np.linalg.solve(D[np.ix_(om, om)], r[om])
        own = (om >= starts[b]) & (om < starts[b + 1])
        z[om[own]] = zl[own]
    assert np.allclose(S.RAS(A, (n, 1, 1), (p, 1, 1), 1).apply(r), z, rtol=1e-13, atol=1e-15)
