"""Pins for the oracle's CPR-type preconditioners (CPR-like Preconditioners
subsection: CPR-FP, CPR-PF, CPR-FPF, CPR-FFPF) and for the aggregation
multigrid V-cycle that stands in for their AMG pressure solve.

The multigrid is pinned by the definitions it is built from, written in
matrix form: Galerkin operators P^T A P with P built here from the aggregate
map; one red-black Gauss-Seidel sweep as a triangular solve in the
red-black ordering; the cycle's error propagation operator by the classical
recursion E_l = S_post (I - P (I - E_{l+1}) A_{l+1}^-1 P^T A) S_pre with
E_L = 0 (the coarsest level exact); an exact solve when one level suffices;
a symmetric cycle for a symmetric matrix.  The CPR stages are pinned by the
decoupling identities, by A_pp = Pi_r W A Pi_p formed densely, by the
pressure residual an exact pressure solve leaves at zero, by the exact
inverse an exact first stage gives, and by the product form of each
algorithm's error propagation operator.  No GPU needed."""
import itertools

import numpy as np
import pytest

import oracle as O
from oracle import cpr as C
from oracle import scalar as S
from paper_1602_05901_amd import inputs as I

OFF = [(0, 0, -1), (0, -1, 0), (-1, 0, 0), (0, 0, 0), (1, 0, 0), (0, 1, 0), (0, 0, 1)]


def laplacian(dims, sigma=0.0, seed=0):
    cfg = I.GenConfig(*dims, I.LNK_IID, sigma, 0.0, 0.0, 0, 1e3, 1.0, seed)
    return S.CSR(*dims, I.poisson(cfg, I.lnk(cfg) if sigma > 0 else None))


def nonsymmetric(dims, seed=0):
    """A 7-point M-matrix with independent coefficients per direction:
    off-diagonals -U(0.1, 1), diagonal = their sum + U(1, 2)."""
    rng = np.random.default_rng(seed)
    nx, ny, nz = dims
    coef = np.zeros((nx * ny * nz, 7))
    for k, j, i in itertools.product(range(nz), range(ny), range(nx)):
        c = i + nx * (j + ny * k)
        for s, (di, dj, dk) in enumerate(OFF):
            if s != 3 and 0 <= i + di < nx and 0 <= j + dj < ny and 0 <= k + dk < nz:
                coef[c, s] = -rng.uniform(0.1, 1.0)
        coef[c, 3] = -coef[c].sum() + rng.uniform(1.0, 2.0)
    return S.CSR(*dims, coef)


def agg_matrix(dims):
    """P[i, agg(i)] = 1 for 2x2x2 aggregation (an axis of one cell kept)."""
    nx, ny, nz = dims
    cx, cy, cz = [(v + 1) // 2 if v > 1 else 1 for v in dims]
    P = np.zeros((nx * ny * nz, cx * cy * cz))
    for k, j, i in itertools.product(range(nz), range(ny), range(nx)):
        P[i + nx * (j + ny * k), (i // 2) + cx * ((j // 2) + cy * (k // 2))] = 1.0
    return P, (cx, cy, cz)


def colours(dims):
    nx, ny, nz = dims
    return np.array([(i + j + k) % 2 for k, j, i in itertools.product(range(nz), range(ny), range(nx))])


def gs_operator(A, dims, first):
    """Matrix G of one Gauss-Seidel sweep from zero over colour `first`, then
    the other: x_new = x + G (b - A x), G = (D + L)^-1 in the ordering that
    lists colour `first` before the other (ascending index within each)."""
    col = colours(dims)
    order = np.concatenate([np.flatnonzero(col == first), np.flatnonzero(col != first)])
    Ap = A[np.ix_(order, order)]
    G = np.linalg.inv(np.tril(Ap))
    out = np.zeros_like(A)
    out[np.ix_(order, order)] = G
    return out


def mg_error_operator(mats, dims_list, Ps, pre, post):
    """E_0 by the two-grid recursion over the given level matrices."""
    L = len(mats)
    E = np.zeros_like(mats[-1])
    for lv in range(L - 2, -1, -1):
        A, d, P, Ac = mats[lv], dims_list[lv], Ps[lv], mats[lv + 1]
        n = A.shape[0]
        Id = np.eye(n)
        Spre = Id - gs_operator(A, d, 0) @ A
        Spost = Id - gs_operator(A, d, 1) @ A
        coarse = P @ (np.eye(Ac.shape[0]) - E) @ np.linalg.solve(Ac, P.T @ A)
        E = np.linalg.matrix_power(Spost, post) @ (Id - coarse) @ np.linalg.matrix_power(Spre, pre)
    return E


def operator_of(apply, n):
    return np.column_stack([apply(e) for e in np.eye(n)])


# ---------------------------------------------------------------- multigrid


@pytest.mark.parametrize("dims", [(9, 6, 5), (8, 1, 4), (1, 1, 13), (2, 2, 2)])
def test_levels_are_galerkin_products_on_halved_grids(dims):
    A = nonsymmetric(dims, 1)
    M = C.MG(A, dims, coarse_max=1)
    lv = M.levels()
    expect = [tuple(dims)]
    while np.prod(expect[-1]) > 1:
        expect.append(tuple((v + 1) // 2 if v > 1 else 1 for v in expect[-1]))
    assert lv == expect
    for l in range(len(lv) - 1):
        P, cdims = agg_matrix(lv[l])
        assert cdims == lv[l + 1]
        Af, Ac = M.level_dense(l), M.level_dense(l + 1)
        assert np.allclose(Ac, P.T @ Af @ P, rtol=1e-14, atol=1e-13)
        # still a 7-point stencil on the coarse grid
        cx, cy, cz = cdims
        for r, c in zip(*np.nonzero(Ac)):
            ri, rj, rk = r % cx, (r // cx) % cy, r // (cx * cy)
            ci, cj, ck = c % cx, (c // cx) % cy, c // (cx * cy)
            assert abs(ri - ci) + abs(rj - cj) + abs(rk - ck) <= 1


def test_coarsening_stops_at_coarse_max():
    A = laplacian((16, 16, 8))
    assert C.MG(A, (16, 16, 8), coarse_max=2048).levels() == [(16, 16, 8)]
    assert C.MG(A, (16, 16, 8), coarse_max=256).levels() == [(16, 16, 8), (8, 8, 4)]
    assert C.MG(A, (16, 16, 8), coarse_max=255).levels() == [(16, 16, 8), (8, 8, 4), (4, 4, 2)]


@pytest.mark.parametrize("dims", [(5, 4, 3), (6, 1, 1), (3, 3, 3)])
@pytest.mark.parametrize("colour", [0, 1])
def test_one_colour_sweep_is_a_triangular_solve(dims, colour):
    A = nonsymmetric(dims, 2)
    Ad = A.dense()
    M = C.MG(A, dims, coarse_max=1)
    rng = np.random.default_rng(3)
    b, x0 = rng.standard_normal(Ad.shape[0]), rng.standard_normal(Ad.shape[0])
    x = M.gs_sweep(b, x0, colour)
    mask = colours(dims) == colour
    # the rows of that colour solve their equations with the other colour fixed
    Dc = Ad[np.ix_(mask, mask)]
    assert np.allclose(Dc, np.diag(np.diag(Dc)))          # no couplings inside a colour
    rhs = b[mask] - Ad[np.ix_(mask, ~mask)] @ x0[~mask]
    assert np.allclose(x[mask], rhs / np.diag(Dc), rtol=1e-13, atol=1e-14)
    assert np.array_equal(x[~mask], x0[~mask])
    # a sweep of both colours from x0 = x0 + G (b - A x0)
    y = M.gs_sweep(b, M.gs_sweep(b, x0, colour), 1 - colour)
    G = gs_operator(Ad, dims, colour)
    assert np.allclose(y, x0 + G @ (b - Ad @ x0), rtol=1e-12, atol=1e-12)


@pytest.mark.parametrize("dims,coarse_max,pre,post", [((6, 5, 4), 60, 1, 1), ((6, 5, 4), 60, 2, 1),
                                                       ((7, 6, 5), 12, 1, 2), ((8, 4, 4), 1, 1, 1),
                                                       ((9, 1, 1), 1, 1, 1)])
@pytest.mark.parametrize("kind", ["laplacian", "nonsymmetric"])
def test_cycle_error_operator_matches_the_multigrid_recursion(dims, coarse_max, pre, post, kind):
    A = laplacian(dims, 1.0, 4) if kind == "laplacian" else nonsymmetric(dims, 5)
    M = C.MG(A, dims, coarse_max=coarse_max, pre=pre, post=post)
    lv = M.levels()
    assert len(lv) >= 2
    mats = [M.level_dense(l) for l in range(len(lv))]
    Ps = [agg_matrix(lv[l])[0] for l in range(len(lv) - 1)]
    n = mats[0].shape[0]
    Minv = operator_of(M.apply, n)
    E = np.eye(n) - Minv @ mats[0]
    Eref = mg_error_operator(mats, lv, Ps, pre, post)
    assert np.max(np.abs(E - Eref)) <= 1e-11


def test_one_level_is_an_exact_solve():
    dims = (5, 4, 3)
    A = nonsymmetric(dims, 6)
    M = C.MG(A, dims, coarse_max=60)
    assert M.levels() == [dims]
    b = np.random.default_rng(7).standard_normal(60)
    assert np.allclose(M.apply(b), np.linalg.solve(A.dense(), b), rtol=1e-13, atol=1e-14)


@pytest.mark.parametrize("pre,post", [(1, 1), (2, 2)])
def test_cycle_is_symmetric_for_a_symmetric_matrix(pre, post):
    dims = (8, 6, 4)
    A = laplacian(dims, 1.5, 8)
    Ad = A.dense()
    assert np.allclose(Ad, Ad.T)
    Minv = operator_of(C.MG(A, dims, coarse_max=8, pre=pre, post=post).apply, Ad.shape[0])
    assert np.max(np.abs(Minv - Minv.T)) <= 1e-13 * np.max(np.abs(Minv))
    # and positive definite
    assert np.min(np.linalg.eigvalsh(0.5 * (Minv + Minv.T))) > 0


def test_cycle_contracts_the_error_of_the_laplacian():
    dims = (16, 16, 16)
    A = laplacian(dims)
    M = C.MG(A, dims, coarse_max=8)
    rng = np.random.default_rng(9)
    x = rng.standard_normal(A.n)
    b = np.zeros(A.n)
    e0 = np.linalg.norm(x)
    for _ in range(10):
        x = x + M.apply(b - A.spmv(x))
    # the V-cycle of unsmoothed aggregation is a contraction (rate < 0.8 here)
    assert np.linalg.norm(x) < 0.8 ** 10 * e0


# ---------------------------------------------------------------- CPR


def block_system(dims, shift=2.0, seed=0, sigma=1.0):
    cfg = I.GenConfig(*dims, I.LNK_IID, sigma, 0.0, shift, 0, 1e3, 1.0, seed)
    B = I.blocks(cfg)
    return cfg, B, O.BCSR.from_stencil(*dims, B)


def dense_blocks(Ao):
    rp, col, val = Ao.export()
    n = Ao.n
    D = np.zeros((3 * n, 3 * n))
    for c in range(n):
        for q in range(rp[c], rp[c + 1]):
            D[3 * c:3 * c + 3, 3 * col[q]:3 * col[q] + 3] = val[q]
    return D


@pytest.mark.parametrize("shift", [2.0, 0.0])
def test_decoupling_weights(shift):
    dims = (4, 3, 3)
    _, B, Ao = block_system(dims, shift, 1)
    R = O.ILU(Ao)
    for dec in (C.DECOUPLE_NONE, C.DECOUPLE_QUASI_IMPES, C.DECOUPLE_ABF):
        w = C.CPR(Ao, dims, R, decouple=dec).weights()
        for c in range(Ao.n):
            D = B[c, 3]
            wd = w[c] @ D
            if dec == C.DECOUPLE_NONE:
                assert np.array_equal(w[c], [1.0, 0.0, 0.0])
            elif dec == C.DECOUPLE_QUASI_IMPES:
                assert w[c, 0] == 1.0
                assert np.all(np.abs(wd[1:]) <= 1e-13 * np.abs(D).max())
            else:
                assert np.allclose(wd, [1.0, 0.0, 0.0], atol=1e-13)


@pytest.mark.parametrize("dec", [0, 1, 2])
def test_pressure_matrix_is_the_restricted_decoupled_matrix(dec):
    dims = (4, 3, 2)
    _, _, Ao = block_system(dims, 2.0, 2)
    P = C.CPR(Ao, dims, O.ILU(Ao), decouple=dec)
    w = P.weights()
    n = Ao.n
    W = np.zeros((n, 3 * n))
    for c in range(n):
        W[c, 3 * c:3 * c + 3] = w[c]
    Pi_p = np.zeros((3 * n, n))
    Pi_p[3 * np.arange(n), np.arange(n)] = 1.0
    App = W @ dense_blocks(Ao) @ Pi_p
    assert np.allclose(P.pressure_dense(), App, rtol=1e-14, atol=1e-14)


@pytest.mark.parametrize("dec", [0, 1, 2])
def test_exact_pressure_solve_leaves_no_pressure_residual(dec):
    dims = (5, 4, 3)
    _, _, Ao = block_system(dims, 0.0, 3)
    P = C.CPR(Ao, dims, O.RAS(Ao, dims, (2, 2, 1), 1), variant=C.FP, decouple=dec, coarse_max=60)
    w = P.weights()
    f = I.test_vector(3, 3 * Ao.n)
    r = (f - Ao.spmv(P.apply(f))).reshape(-1, 3)
    assert np.max(np.abs((w * r).sum(axis=1))) <= 1e-12 * np.abs(f).max()


@pytest.mark.parametrize("dims", [(12, 1, 1), (1, 1, 9)])
@pytest.mark.parametrize("variant", [C.FP, C.PF, C.FPF, C.FFPF])
def test_exact_first_stage_gives_the_exact_inverse(dims, variant):
    _, _, Ao = block_system(dims, 0.0, 4)
    # on a line of cells ILU(0) is the exact LU, so R^-1 = A^-1
    P = C.CPR(Ao, dims, O.ILU(Ao), variant=variant, decouple=C.DECOUPLE_QUASI_IMPES, coarse_max=2)
    f = I.test_vector(4, 3 * Ao.n)
    x = np.linalg.solve(dense_blocks(Ao), f)
    assert np.allclose(P.apply(f), x, rtol=1e-11, atol=1e-12 * np.abs(x).max())


@pytest.mark.parametrize("variant", [C.FP, C.PF, C.FPF, C.FFPF])
@pytest.mark.parametrize("dec", [0, 1])
def test_error_propagation_is_the_product_of_the_stages(variant, dec):
    dims = (4, 3, 3)
    _, _, Ao = block_system(dims, 0.0, 5)
    n = Ao.n
    R = O.RAS(Ao, dims, (2, 1, 1), 1)
    P = C.CPR(Ao, dims, R, variant=variant, decouple=dec, coarse_max=4)
    A = dense_blocks(Ao)
    MR = operator_of(R.apply, 3 * n)
    # the pressure stage as an operator: Pi_p M_g Pi_r W, with M_g the same
    # V-cycle built again from the pressure matrix
    w = P.weights()
    mg = C.MG(S.CSR.from_arrays(*P.pressure_csr(), dims), dims, coarse_max=4)
    Mg = operator_of(mg.apply, n)
    W = np.zeros((n, 3 * n))
    for c in range(n):
        W[c, 3 * c:3 * c + 3] = w[c]
    Pi_p = np.zeros((3 * n, n))
    Pi_p[3 * np.arange(n), np.arange(n)] = 1.0
    MP = Pi_p @ Mg @ W
    Id = np.eye(3 * n)
    ER, EP = Id - MR @ A, Id - MP @ A
    expect = {C.FP: EP @ ER, C.PF: ER @ EP, C.FPF: ER @ EP @ ER, C.FFPF: ER @ EP @ ER @ ER}[variant]
    E = Id - operator_of(P.apply, 3 * n) @ A
    assert np.max(np.abs(E - expect)) <= 1e-10 * max(1.0, np.max(np.abs(expect)))


def test_setup_errors():
    dims = (3, 3, 2)
    _, B, Ao = block_system(dims, 2.0, 6)
    with pytest.raises(O.OracleError):
        C.CPR(Ao, (3, 3, 3), O.ILU(Ao))
    with pytest.raises(O.OracleError):
        C.CPR(Ao, dims, O.ILU(Ao), variant=4)
    # a diagonal block whose saturation part is singular: quasi-IMPES fails at that cell
    B2 = B.copy()
    B2[7, 3][1:, 1:] = [[1.0, 2.0], [2.0, 4.0]]
    Ao2 = O.BCSR.from_stencil(*dims, B2)
    with pytest.raises(O.OracleError) as e:
        C.CPR(Ao2, dims, O.RAS(Ao, dims, (1, 1, 1), 0), decouple=C.DECOUPLE_QUASI_IMPES)
    assert e.value.rc == O.ERR_ZERO_PIVOT and e.value.bad_cell == 7


def test_cpr_reduces_gmres_steps_on_the_literal_reading():
    cfg = I.preset("C1", seed=0)            # literal coupling matrices
    B = I.blocks(cfg)
    dims = (cfg.nx, cfg.ny, cfg.nz)
    Ao = O.BCSR.from_stencil(*dims, B)
    b = Ao.spmv(I.x_true(cfg))
    R = O.RAS(Ao, dims, (2, 2, 2), 1)
    its_r = O.gmres(Ao, b, pc=R, m=30, tol=1e-8, maxit=3000)["its"]
    out = O.gmres(Ao, b, pc=C.CPR(Ao, dims, R, variant=C.FPF), m=30, tol=1e-8, maxit=3000)
    assert out["rc"] == 0 and out["relres"] <= 1e-8
    assert out["its"] < its_r / 2
