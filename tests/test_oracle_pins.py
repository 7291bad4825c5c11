"""Pins for the CPU oracle: each test checks it against something other than
itself -- brute-force dense algebra, closed forms, invariants of the input
recipe, and special cases that reduce to textbook results.  No GPU needed.
"""
import numpy as np
import pytest

from paper_1602_05901_amd import inputs as I
import oracle as O

OFF = [(0, 0, -1), (0, -1, 0), (-1, 0, 0), (0, 0, 0), (1, 0, 0), (0, 1, 0), (0, 0, 1)]


def dense_from_blocks(nx, ny, nz, B):
    """Dense matrix assembled directly from the stencil blocks (independent of
    the oracle's block-CSR code)."""
    n = nx * ny * nz
    D = np.zeros((3 * n, 3 * n))
    for k in range(nz):
        for j in range(ny):
            for i in range(nx):
                c = i + nx * (j + ny * k)
                for s, (di, dj, dk) in enumerate(OFF):
                    ii, jj, kk = i + di, j + dj, k + dk
                    if 0 <= ii < nx and 0 <= jj < ny and 0 <= kk < nz:
                        m = ii + nx * (jj + ny * kk)
                        D[3 * c:3 * c + 3, 3 * m:3 * m + 3] = B[c, s]
    return D


def small(nx, ny, nz, seed=0, shift=2.0, sigma=1.0, nsrc=0):
    cfg = I.GenConfig(nx, ny, nz, I.LNK_IID, sigma, 0.0, shift, nsrc, 1e3, 1.0, seed)
    B = I.blocks(cfg)
    return cfg, B, O.BCSR.from_stencil(nx, ny, nz, B)


def factors_dense(F, n):
    rp, col, val = F.factors()
    L = np.eye(3 * n)
    U = np.zeros((3 * n, 3 * n))
    for i in range(n):
        for p in range(rp[i], rp[i + 1]):
            j = col[p]
            if j < i:
                L[3 * i:3 * i + 3, 3 * j:3 * j + 3] = val[p]
            else:
                U[3 * i:3 * i + 3, 3 * j:3 * j + 3] = val[p]
    return L, U, rp, col


# ---------------------------------------------------------------- inputs / SpMV

def test_generator_deterministic_and_recipe():
    cfg = I.preset("C1", seed=3)
    a = I.blocks(cfg)
    b = I.blocks(cfg)
    assert np.array_equal(a, b)
    # absent neighbours are zero blocks: cell 0 has no -x,-y,-z neighbours
    assert np.all(a[0, 0:3] == 0)
    # off-diagonal block = -T * M with M entries in [0.1, 1) + shift*I, T > 0
    blk = a[1, 2]               # cell 1, -x neighbour (cell 0)
    lk = I.lnk(cfg)
    ka, kb = np.exp(lk[1]), np.exp(lk[0])
    T = 2 * ka * kb / (ka + kb)
    M = -blk / T
    off = M - np.diag(np.diag(M))
    assert np.all((off[off != 0] >= 0.1) & (off[off != 0] < 1.0))
    d = np.diag(M) - cfg.m_shift
    assert np.all((d >= 0.1) & (d < 1.0))


def test_lognormal_std_reading():
    # ln k ~ N(0, sigma) with sigma the standard deviation
    cfg = I.GenConfig(64, 64, 16, I.LNK_IID, 3.0, 0.0, 2.0, 0, 1e3, 1.0, 7)
    lk = I.lnk(cfg)
    assert abs(lk.std() - 3.0) < 0.05 and abs(lk.mean()) < 0.05


def test_spmv_vs_dense():
    for dims in [(3, 2, 2), (4, 3, 2), (1, 1, 5), (5, 1, 1)]:
        cfg, B, A = small(*dims, seed=1)
        D = dense_from_blocks(*dims, B)
        x = I.test_vector(11, D.shape[0])
        y = A.spmv(x)
        assert np.allclose(y, D @ x, rtol=0, atol=1e-14 * np.abs(D).sum(1).max() * np.abs(x).max())


def test_spmv_invariant_A_times_ones_is_accumulation():
    for name, shift in [("C1", 0.0), ("C1", 2.0)]:
        cfg = I.preset(name, seed=0, m_shift=shift)
        B = I.blocks(cfg)
        A = O.BCSR.from_stencil(cfg.nx, cfg.ny, cfg.nz, B)
        acc = I.accumulation(cfg)
        y = A.spmv(np.ones(3 * cfg.ncell))
        scale = np.abs(B[:, 3]).max()
        assert np.abs(y - acc).max() <= 1e-12 * scale
    # sources add 1e3 to their three scalar diagonal entries
    cfg = I.GenConfig(6, 5, 4, I.LNK_LAYERED, 2.0, 1.5, 2.0, 4, 1e3, 1.0, 5)
    B = I.blocks(cfg)
    A = O.BCSR.from_stencil(cfg.nx, cfg.ny, cfg.nz, B)
    y = A.spmv(np.ones(3 * cfg.ncell)).reshape(-1, 3)
    src = I.source_cells(cfg)
    assert len(src) == 4
    assert np.all(y[src] > 1e3) and np.all(np.delete(y, src, axis=0) < 10.0 + 1e-9)


def test_pattern_error():
    cfg, B, _ = small(3, 3, 3)
    B = B.copy()
    B[0, 2, 0, 0] = 1.0   # -x slot of cell 0 lies outside the grid
    with pytest.raises(O.OracleError) as e:
        O.BCSR.from_stencil(3, 3, 3, B)
    assert e.value.rc == O.ERR_PATTERN


# ---------------------------------------------------------------- 3x3 inverse

def test_inv3():
    rng = np.random.default_rng(0)
    for _ in range(50):
        a = rng.standard_normal((3, 3))
        rc, ai = O.inv3(a)
        assert rc == 0
        assert np.allclose(ai, np.linalg.inv(a), rtol=1e-12, atol=1e-12 * np.abs(np.linalg.inv(a)).max())
    rc, _ = O.inv3(np.zeros((3, 3)))
    assert rc == O.ERR_ZERO_PIVOT
    rc, _ = O.inv3(np.array([[1, 2, 3], [2, 4, 6], [1, 0, 1.0]]))
    assert rc == O.ERR_ZERO_PIVOT


# ---------------------------------------------------------------- ILU(0)

def test_ilu0_matches_A_on_pattern():
    """ILU(0) characterisation: (LU)_ij = A_ij for every (i,j) in the pattern."""
    dims = (4, 3, 2)
    cfg, B, A = small(*dims, seed=2, shift=0.0)
    n = cfg.ncell
    D = dense_from_blocks(*dims, B)
    L, U, rp, col = factors_dense(O.ILU(A), n)
    LU = L @ U
    mask = np.zeros((n, n), bool)
    for i in range(n):
        mask[i, col[rp[i]:rp[i + 1]]] = True
    M = np.kron(mask, np.ones((3, 3), bool))
    err = np.abs(LU - D)[M].max()
    assert err <= 1e-13 * np.abs(D).max()
    # and the factorisation is genuinely incomplete off the pattern
    assert np.abs(LU - D)[~M].max() > 1e-6


def test_ilu0_exact_on_1d_grid():
    """A 1-D grid gives a block-tridiagonal A, whose ILU(0) is its exact LU."""
    for dims in [(7, 1, 1), (1, 6, 1), (1, 1, 8)]:
        cfg, B, A = small(*dims, seed=4, shift=0.0, sigma=2.0)
        D = dense_from_blocks(*dims, B)
        L, U, _, _ = factors_dense(O.ILU(A), cfg.ncell)
        assert np.abs(L @ U - D).max() <= 1e-13 * np.abs(D).max()


def test_ilu0_two_cell_hand_case():
    cfg, B, A = small(2, 1, 1, seed=5)
    A00, A01, A10, A11 = B[0, 3], B[0, 4], B[1, 2], B[1, 3]
    rp, col, val = O.ILU(A).factors()
    # row 0: U00 = A00, U01 = A01 ; row 1: L10 = A10 A00^-1, U11 = A11 - A10 A00^-1 A01
    assert np.allclose(val[0], A00, rtol=0, atol=0)
    assert np.allclose(val[1], A01, rtol=0, atol=0)
    inv = np.linalg.inv(A00)
    assert np.allclose(val[2], A10 @ inv, rtol=1e-13)
    assert np.allclose(val[3], A11 - A10 @ inv @ A01, rtol=1e-13)


def test_ilu0_diagonal_closed_form():
    """On the bipartite 7-point graph the pivots satisfy
    D_c = A_cc - sum_{k in {-x,-y,-z}} A_ck D_k^{-1} A_kc (ascending c)."""
    dims = (4, 3, 3)
    nx, ny, nz = dims
    cfg, B, A = small(*dims, seed=6, shift=0.0, sigma=1.5)
    rp, col, val = O.ILU(A).factors()
    n = cfg.ncell
    Dblk = np.zeros((n, 3, 3))
    for c in range(n):
        i, j, k = c % nx, (c // nx) % ny, c // (nx * ny)
        d = B[c, 3].copy()
        for s, (di, dj, dk) in enumerate(OFF[:3]):
            ii, jj, kk = i + di, j + dj, k + dk
            if ii >= 0 and jj >= 0 and kk >= 0:
                m = ii + nx * (jj + ny * kk)
                up = {0: 6, 1: 5, 2: 4}[s]
                d -= B[c, s] @ np.linalg.solve(Dblk[m], B[m, up])
        Dblk[c] = d
        p = [q for q in range(rp[c], rp[c + 1]) if col[q] == c][0]
        assert np.allclose(val[p], d, rtol=1e-12, atol=1e-12 * np.abs(d).max())


def test_ilu_apply_is_dense_LU_solve():
    for dims in [(4, 3, 2), (3, 3, 3)]:
        cfg, B, A = small(*dims, seed=7, shift=0.0)
        F = O.ILU(A)
        L, U, _, _ = factors_dense(F, cfg.ncell)
        r = I.test_vector(3, 3 * cfg.ncell)
        z = F.apply(r)
        zd = np.linalg.solve(L @ U, r)
        assert np.linalg.norm(z - zd) <= 1e-13 * np.linalg.norm(zd) * 10


def test_ilu_fp32_apply():
    """FP32 sweeps: within FP32 rounding of a dense FP32 triangular solve with the
    rounded factors, and about 1e-7 relative from the FP64 apply."""
    cfg, B, A = small(4, 4, 3, seed=8, shift=2.0, sigma=2.0)
    F = O.ILU(A)
    L, U, _, _ = factors_dense(F, cfg.ncell)
    r = I.test_vector(4, 3 * cfg.ncell)
    z32 = F.apply(r, fp32=True)
    z64 = F.apply(r)
    rel = np.linalg.norm(z32 - z64) / np.linalg.norm(z64)
    assert 1e-10 < rel < 1e-5
    import scipy.linalg as sl
    y = sl.solve_triangular(L.astype(np.float32), r.astype(np.float32), lower=True, unit_diagonal=True)
    zd = np.linalg.solve(U.astype(np.float32), y)   # block upper: full 3x3 diagonal blocks
    assert zd.dtype == np.float32
    assert np.linalg.norm(z32 - zd) / np.linalg.norm(zd) < 1e-5


def test_zero_pivot_detected():
    cfg, B, _ = small(3, 3, 2, seed=9)
    B = B.copy()
    B[4, 3] = 0.0          # singular diagonal block at cell 4 (no lower coupling can fix it for row 0)
    B[0, 3] = 0.0
    A = O.BCSR.from_stencil(3, 3, 2, B)
    with pytest.raises(O.OracleError) as e:
        O.ILU(A)
    assert e.value.rc == O.ERR_ZERO_PIVOT and e.value.bad_cell == 0


# ---------------------------------------------------------------- RAS

def test_ras_one_subdomain_is_ilu():
    cfg, B, A = small(5, 4, 3, seed=10)
    r = I.test_vector(5, 3 * cfg.ncell)
    z1 = O.RAS(A, (5, 4, 3), (1, 1, 1), 1).apply(r)
    z0 = O.ILU(A).apply(r)
    assert np.linalg.norm(z1 - z0) <= 1e-15 * np.linalg.norm(z0) * 10


def test_ras_large_overlap_is_ilu():
    cfg, B, A = small(4, 3, 3, seed=11)
    r = I.test_vector(6, 3 * cfg.ncell)
    R = O.RAS(A, (4, 3, 3), (2, 2, 1), 10)   # overlap >= graph diameter
    for s in range(R.nsub):
        assert len(R.sub_cells(s)) == cfg.ncell
    z0 = O.ILU(A).apply(r)
    assert np.linalg.norm(R.apply(r) - z0) <= 1e-14 * np.linalg.norm(z0)


def test_ras_overlap0_is_block_jacobi_ilu():
    dims = (6, 4, 2)
    nx, ny, nz = dims
    cfg, B, A = small(*dims, seed=12)
    R = O.RAS(A, dims, (2, 2, 1), 0)
    owner = R.owner()
    B2 = B.copy()
    for c in range(cfg.ncell):
        i, j, k = c % nx, (c // nx) % ny, c // (nx * ny)
        for s, (di, dj, dk) in enumerate(OFF):
            ii, jj, kk = i + di, j + dj, k + dk
            if s != 3 and 0 <= ii < nx and 0 <= jj < ny and 0 <= kk < nz:
                if owner[ii + nx * (jj + ny * kk)] != owner[c]:
                    B2[c, s] = 0.0
    A2 = O.BCSR.from_stencil(*dims, B2)
    r = I.test_vector(7, 3 * cfg.ncell)
    z0 = O.ILU(A2).apply(r)
    assert np.linalg.norm(R.apply(r) - z0) <= 1e-14 * np.linalg.norm(z0)


def test_ras_singletons_is_pointblock_jacobi():
    dims = (3, 2, 2)
    cfg, B, A = small(*dims, seed=13)
    R = O.RAS(A, dims, dims, 0)
    r = I.test_vector(8, 3 * cfg.ncell)
    z = R.apply(r).reshape(-1, 3)
    ref = np.stack([np.linalg.solve(B[c, 3], r.reshape(-1, 3)[c]) for c in range(cfg.ncell)])
    assert np.abs(z - ref).max() <= 1e-13 * np.abs(ref).max()


def test_ras_overlap_geometry_and_exact_local_solves():
    """1-D grid: local ILU(0) is exact, so RAS = sum_s Rt_s^T A_s^{-1} R_s r with
    Omega_s = owned cells plus graph-distance-1 neighbours; checked with dense
    solves.  Also checks the face-only (no edge/corner) overlap on a 3-D grid."""
    dims = (10, 1, 1)
    cfg, B, A = small(*dims, seed=14, shift=0.0)
    D = dense_from_blocks(*dims, B)
    R = O.RAS(A, dims, (3, 1, 1), 1)
    owner = R.owner()
    assert list(owner) == [0, 0, 0, 0, 1, 1, 1, 2, 2, 2]   # first part one longer
    r = I.test_vector(9, 30)
    z = np.zeros(30)
    for s in range(3):
        own = np.where(owner == s)[0]
        omega = sorted(set(own) | {c - 1 for c in own if c > 0} | {c + 1 for c in own if c < 9})
        assert list(R.sub_cells(s)) == omega
        idx = np.concatenate([np.arange(3 * c, 3 * c + 3) for c in omega])
        zl = np.linalg.solve(D[np.ix_(idx, idx)], r[idx])
        for q, c in enumerate(omega):
            if owner[c] == s:
                z[3 * c:3 * c + 3] = zl[3 * q:3 * q + 3]
    assert np.linalg.norm(R.apply(r) - z) <= 1e-13 * np.linalg.norm(z)
    # 3-D: overlap 1 adds face neighbours only
    dims = (6, 6, 4)
    nx, ny, nz = dims
    cfg, B, A = small(*dims, seed=15)
    R = O.RAS(A, dims, (2, 2, 2), 1)
    owner = R.owner()
    for s in range(R.nsub):
        own = set(np.where(owner == s)[0])
        exp = set(own)
        for c in own:
            i, j, k = c % nx, (c // nx) % ny, c // (nx * ny)
            for di, dj, dk in OFF:
                ii, jj, kk = i + di, j + dj, k + dk
                if 0 <= ii < nx and 0 <= jj < ny and 0 <= kk < nz:
                    exp.add(ii + nx * (jj + ny * kk))
        assert set(R.sub_cells(s)) == exp


# ---------------------------------------------------------------- GMRES

def _krylov_min(Dm, b, x0, Minv, j):
    """x0 + M^{-1} K_j(A M^{-1}, r0) minimiser of ||b - A x|| by dense least squares."""
    r0 = b - Dm @ x0
    K = [r0]
    for _ in range(j - 1):
        K.append(Dm @ (Minv @ K[-1]))
    K = np.stack(K, 1)
    # orthonormalise the basis for conditioning (same span)
    Q, _ = np.linalg.qr(K)
    W = Minv @ Q
    c, *_ = np.linalg.lstsq(Dm @ W, r0, rcond=None)
    return x0 + W @ c


def test_gmres_iterates_are_krylov_minimisers():
    dims = (3, 2, 2)
    cfg, B, A = small(*dims, seed=16, shift=0.0, sigma=1.0)
    D = dense_from_blocks(*dims, B)
    F = O.ILU(A)
    L, U, _, _ = factors_dense(F, cfg.ncell)
    Minv = np.linalg.inv(L @ U)
    b = I.test_vector(10, 36)
    x0 = I.test_vector(12, 36) * 0.1
    for j in range(1, 6):
        for pc, Mi in [(None, np.eye(36)), (F, Minv)]:
            out = O.gmres(A, b, pc=pc, x0=x0, m=30, tol=0.0, maxit=j)
            ref = _krylov_min(D, b, x0, Mi, j)
            assert np.linalg.norm(out["x"] - ref) <= 1e-9 * np.linalg.norm(ref), (j, pc)
            assert out["its"] == j


def test_gmres_restarted_iterates():
    """GMRES(m) with restarts: each cycle minimises over its own Krylov space."""
    dims = (3, 2, 2)
    cfg, B, A = small(*dims, seed=17, shift=0.0)
    D = dense_from_blocks(*dims, B)
    b = I.test_vector(13, 36)
    x = np.zeros(36)
    m = 3
    for cycle in range(3):
        x = _krylov_min(D, b, x, np.eye(36), m)
    out = O.gmres(A, b, pc=None, m=m, tol=0.0, maxit=3 * m)
    assert out["restarts"] == 3
    assert np.linalg.norm(out["x"] - x) <= 1e-9 * np.linalg.norm(x)


def test_full_gmres_exact_in_n_steps():
    dims = (2, 2, 1)
    cfg, B, A = small(*dims, seed=18, shift=0.0)
    D = dense_from_blocks(*dims, B)
    n = 12
    b = I.test_vector(14, n)
    out = O.gmres(A, b, pc=None, m=n, tol=1e-12, maxit=n)
    assert out["rc"] == O.OK and out["its"] <= n
    assert np.linalg.norm(out["x"] - np.linalg.solve(D, b)) <= 1e-9 * np.linalg.norm(out["x"])


def test_gmres_exact_preconditioner_one_step():
    dims = (9, 1, 1)
    cfg, B, A = small(*dims, seed=19, shift=0.0, sigma=2.0)
    b = A.spmv(I.x_true(cfg))
    out = O.gmres(A, b, pc=O.ILU(A), m=30, tol=1e-10, maxit=50)
    assert out["rc"] == O.OK and out["its"] == 1


def test_gmres_manufactured_solution_C1():
    for shift in (0.0, 2.0):
        cfg = I.preset("C1", seed=0, m_shift=shift)
        A = O.BCSR.from_stencil(cfg.nx, cfg.ny, cfg.nz, I.blocks(cfg))
        xt = I.x_true(cfg)
        b = A.spmv(xt)
        out = O.gmres(A, b, pc=O.ILU(A), m=30, tol=1e-8, maxit=3000, hist=True)
        assert out["rc"] == O.OK and out["relres"] <= 1e-8
        assert np.linalg.norm(b - A.spmv(out["x"])) / np.linalg.norm(b) <= 1e-8
        assert np.linalg.norm(out["x"] - xt) / np.linalg.norm(xt) <= 1e-5
        assert out["hist"][0] == pytest.approx(1.0)


def test_gmres_edge_cases():
    cfg, B, A = small(3, 3, 2, seed=20)
    n = 3 * cfg.ncell
    out = O.gmres(A, np.zeros(n), pc=None)
    assert out["rc"] == O.OK and np.all(out["x"] == 0)
    bad = np.ones(n)
    bad[5] = np.nan
    assert O.gmres(A, bad)["rc"] == O.ERR_NAN
    out = O.gmres(A, np.ones(n), pc=None, m=5, tol=1e-14, maxit=3)
    assert out["rc"] == O.NOT_CONVERGED and out["its"] == 3


# ---------------------------------------------------------------- BiCGSTAB

def test_bicgstab_first_iteration_properties():
    """One iteration: alpha from the Galerkin condition r0 . s = 0, omega
    minimising ||s - omega t||."""
    dims = (3, 2, 2)
    cfg, B, A = small(*dims, seed=21, shift=0.0)
    D = dense_from_blocks(*dims, B)
    F = O.ILU(A)
    L, U, _, _ = factors_dense(F, cfg.ncell)
    Minv = np.linalg.inv(L @ U)
    b = I.test_vector(15, 36)
    out = O.bicgstab(A, b, pc=F, tol=0.0, maxit=1)
    r0 = b
    AM = D @ Minv
    alpha = (r0 @ r0) / (r0 @ (AM @ r0))
    s = r0 - alpha * AM @ r0
    assert abs(r0 @ s) <= 1e-12 * np.linalg.norm(r0) * np.linalg.norm(s) * 100
    t = AM @ s
    om, *_ = np.linalg.lstsq(t[:, None], s, rcond=None)
    x1 = Minv @ (alpha * r0 + om[0] * s)
    assert np.linalg.norm(out["x"] - x1) <= 1e-11 * np.linalg.norm(x1)


def test_bicgstab_dense_agreement_and_exact_pc():
    dims = (4, 3, 2)
    cfg, B, A = small(*dims, seed=22, shift=0.0)
    D = dense_from_blocks(*dims, B)
    b = I.test_vector(16, D.shape[0])
    out = O.bicgstab(A, b, pc=O.ILU(A), tol=1e-12, maxit=500)
    xd = np.linalg.solve(D, b)
    assert out["rc"] == O.OK
    assert np.linalg.norm(out["x"] - xd) <= 1e-9 * np.linalg.norm(xd)
    cfg, B, A = small(8, 1, 1, seed=23, sigma=2.0)
    b = A.spmv(I.x_true(cfg))
    out = O.bicgstab(A, b, pc=O.ILU(A), tol=1e-10, maxit=10)
    assert out["rc"] == O.OK and out["its"] == 1


def test_bicgstab_manufactured_C1():
    cfg = I.preset("C1", seed=1, m_shift=2.0)
    A = O.BCSR.from_stencil(cfg.nx, cfg.ny, cfg.nz, I.blocks(cfg))
    xt = I.x_true(cfg)
    b = A.spmv(xt)
    out = O.bicgstab(A, b, pc=O.ILU(A), tol=1e-8, maxit=1000)
    assert out["rc"] == O.OK and out["relres"] <= 1e-8
    assert np.linalg.norm(out["x"] - xt) / np.linalg.norm(xt) <= 1e-6


# ---------------------------------------------------------------- FGMRES

def test_fgmres_with_fixed_pc_equals_gmres():
    cfg = I.preset("C1", seed=2, m_shift=2.0)
    A = O.BCSR.from_stencil(cfg.nx, cfg.ny, cfg.nz, I.blocks(cfg))
    F = O.ILU(A)
    b = A.spmv(I.x_true(cfg))
    g = O.gmres(A, b, pc=F, tol=1e-8, maxit=200, hist=True)
    f = O.fgmres(A, b, pc=F, fallback=F, theta=10.0, tol=1e-8, maxit=200, hist=True)
    assert g["its"] == f["its"] and f["fallbacks"] == 0
    assert np.allclose(g["hist"], f["hist"], rtol=1e-10, atol=1e-14)
    assert np.linalg.norm(g["x"] - f["x"]) <= 1e-9 * np.linalg.norm(g["x"])


def test_fgmres_exact_inverse_one_step_and_fallback():
    dims = (3, 3, 2)
    cfg, B, A = small(*dims, seed=24)
    D = dense_from_blocks(*dims, B)
    Dinv = np.linalg.inv(D)
    F = O.ILU(A)
    b = I.test_vector(17, D.shape[0])
    out = O.fgmres(A, b, pc=lambda v: Dinv @ v, fallback=F, tol=1e-10, maxit=20)
    assert out["rc"] == O.OK and out["its"] == 1 and out["fallbacks"] == 0
    # a preconditioner that returns NaN: every column falls back, still converges
    out = O.fgmres(A, b, pc=lambda v: v * np.nan, fallback=F, tol=1e-10, maxit=200)
    g = O.gmres(A, b, pc=F, tol=1e-10, maxit=200)
    assert out["rc"] == O.OK and out["fallbacks"] == out["its"] and out["its"] == g["its"]
    # a zero preconditioner never reduces the residual: falls back too
    out = O.fgmres(A, b, pc=lambda v: 0 * v, fallback=F, tol=1e-10, maxit=200)
    assert out["rc"] == O.OK and out["fallbacks"] == out["its"]
