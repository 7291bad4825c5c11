"""Pins for the oracle's ILUT(p, tol) with 3x3 blocks (the RAS local solver
named by the RAS parameters' ilut_p and ilut_tol): tol = 0 with room for
every fill block is the exact LU; a tolerance that drops everything, or
p = 0, is block Jacobi; a line of cells (no fill) reproduces ILU(0); the
first two rows by hand (numpy) for several tolerances and p; every kept
block passes the drop test and no row keeps more than p; RAS with ILUT
local solvers reduces to ILUT of the whole grid and to block Jacobi in its
special cases.  No GPU needed."""
import numpy as np
import pytest

import oracle as O
from paper_1602_05901_amd import inputs as I


def system(dims, shift=2.0, seed=0, sigma=1.0):
    cfg = I.GenConfig(*dims, I.LNK_IID, sigma, 0.0, shift, 0, 1e3, 1.0, seed)
    B = I.blocks(cfg)
    return cfg, B, O.BCSR.from_stencil(*dims, B)


def dense_of(rp, col, val, n):
    D = np.zeros((3 * n, 3 * n))
    for i in range(n):
        for q in range(rp[i], rp[i + 1]):
            D[3 * i:3 * i + 3, 3 * col[q]:3 * col[q] + 3] = val[q]
    return D


def lu_product(F, n):
    rp, col, val = F.factors()
    L = np.eye(3 * n)
    U = np.zeros((3 * n, 3 * n))
    for i in range(n):
        for q in range(rp[i], rp[i + 1]):
            blk = (slice(3 * i, 3 * i + 3), slice(3 * col[q], 3 * col[q] + 3))
            (L if col[q] < i else U)[blk] = val[q]
    return L @ U


def fro2(b):
    return float((b * b).sum())


@pytest.mark.parametrize("dims", [(4, 3, 3), (5, 4, 2), (3, 3, 3)])
@pytest.mark.parametrize("shift", [2.0, 0.0])
def test_zero_tolerance_is_the_exact_lu(dims, shift):
    _, _, Ao = system(dims, shift, 1)
    n = Ao.n
    A = dense_of(*Ao.export(), n)
    F = O.ILU(Ao, ilut=(3 * n, 0.0))
    assert np.allclose(lu_product(F, n), A, rtol=0, atol=1e-11 * np.abs(A).max())
    r = I.test_vector(1, 3 * n)
    x = np.linalg.solve(A, r)
    assert np.allclose(F.apply(r), x, rtol=1e-10, atol=1e-12 * np.abs(x).max())


@pytest.mark.parametrize("p,tol", [(-1, 1e300), (5, 1e300), (0, 1e-3), (0, 0.0)])
def test_everything_dropped_is_block_jacobi(p, tol):
    dims = (5, 4, 3)
    _, B, Ao = system(dims, 2.0, 2)
    n = Ao.n
    F = O.ILU(Ao, ilut=(p, tol))
    rp, col, val = F.factors()
    assert np.all(col == np.arange(n)) and np.all(np.diff(rp) == 1)
    assert np.array_equal(val, B[:, 3])
    r = I.test_vector(2, 3 * n).reshape(-1, 3)
    z = np.stack([np.linalg.solve(B[c, 3], r[c]) for c in range(n)])
    assert np.allclose(F.apply(r.reshape(-1)), z.reshape(-1), rtol=1e-12, atol=1e-14)


@pytest.mark.parametrize("dims", [(12, 1, 1), (1, 1, 9), (1, 7, 1)])
def test_a_line_of_cells_is_ilu0(dims):
    _, _, Ao = system(dims, 0.0, 3)
    F0 = O.ILU(Ao)
    F = O.ILU(Ao, ilut=(-1, 1e-12))
    rp0, col0, val0 = F0.factors()
    rp, col, val = F.factors()
    assert np.array_equal(rp, rp0) and np.array_equal(col, col0)
    assert np.allclose(val, val0, rtol=1e-13, atol=1e-15 * np.abs(val0).max())


def expected_first_rows(Ao, p, tol):
    """Rows 0 and 1 of ILUT(p, tol) computed here step by step."""
    rp, col, val = Ao.export()
    n = Ao.n

    def row(i):
        return {int(col[q]): val[q].copy() for q in range(rp[i], rp[i + 1])}

    def keep(cands, w, limit):
        order = sorted(cands, key=lambda j: (-fro2(w[j]), j))
        return sorted(order[:limit])

    out = []
    U0 = None
    for i in (0, 1):
        w = row(i)
        a_row = row(i)
        thr = tol * tol * sum(fro2(b) for b in a_row.values())
        nla = sum(1 for j in a_row if j < i)
        nua = sum(1 for j in a_row if j > i)
        Lkept = {}
        if i == 1 and 0 in w:
            w0 = w[0] @ np.linalg.inv(U0[0])
            if not fro2(w0) < thr:
                w[0] = w0
                for j, b in U0.items():
                    if j > 0:
                        w[j] = w.get(j, np.zeros((3, 3))) - w0 @ b
                Lkept = {0: w0}
            else:
                del w[0]
        lsel = keep([j for j in Lkept], w, nla if p < 0 else p)
        ucand = [j for j in w if j > i and not fro2(w[j]) < thr]
        usel = keep(ucand, w, nua if p < 0 else p)
        U = {i: w[i]}
        U.update({j: w[j] for j in usel})
        out.append(({j: w[j] for j in lsel}, U))
        if i == 0:
            U0 = U
    return out


@pytest.mark.parametrize("p", [-1, 1, 2, 5])
@pytest.mark.parametrize("tol", [0.0, 0.05, 0.15, 0.3, 0.6])
def test_first_two_rows_by_hand(p, tol):
    dims = (4, 3, 2)
    _, _, Ao = system(dims, 2.0, 4)
    F = O.ILU(Ao, ilut=(p, tol))
    rp, col, val = F.factors()
    for i, (Lexp, Uexp) in enumerate(expected_first_rows(Ao, p, tol)):
        got = {int(col[q]): val[q] for q in range(rp[i], rp[i + 1])}
        exp = dict(Lexp)
        exp.update(Uexp)
        assert sorted(got) == sorted(exp), (i, sorted(got), sorted(exp))
        for j in exp:
            assert np.allclose(got[j], exp[j], rtol=1e-13, atol=1e-14 * np.abs(exp[j]).max())


@pytest.mark.parametrize("dims,shift", [((6, 5, 4), 2.0), ((6, 5, 4), 0.0), ((20, 20, 10), 0.0)])
@pytest.mark.parametrize("p,tol", [(-1, 1e-3), (2, 1e-2), (6, 1e-4)])
def test_kept_blocks_pass_the_drop_test_and_the_count(dims, shift, p, tol):
    _, _, Ao = system(dims, shift, 5)
    n = Ao.n
    rpa, cola, vala = Ao.export()
    F = O.ILU(Ao, ilut=(p, tol))
    rp, col, val = F.factors()
    for i in range(n):
        thr = tol * tol * sum(fro2(vala[q]) for q in range(rpa[i], rpa[i + 1]))
        nla = sum(1 for q in range(rpa[i], rpa[i + 1]) if cola[q] < i)
        nua = sum(1 for q in range(rpa[i], rpa[i + 1]) if cola[q] > i)
        cols = col[rp[i]:rp[i + 1]]
        assert np.all(np.diff(cols) > 0) and i in cols
        nl = int((cols < i).sum())
        nu = int((cols > i).sum())
        assert nl <= (nla if p < 0 else p) and nu <= (nua if p < 0 else p)
        for q in range(rp[i], rp[i + 1]):
            if col[q] != i:
                assert fro2(val[q]) >= thr


def test_smaller_tolerance_approximates_better():
    dims = (6, 5, 4)
    _, _, Ao = system(dims, 0.0, 6)
    n = Ao.n
    A = dense_of(*Ao.export(), n)
    err = [np.linalg.norm(lu_product(O.ILU(Ao, ilut=(3 * n, t)), n) - A) for t in (1e-1, 1e-2, 1e-4, 0.0)]
    assert err[0] > err[2] and err[1] > err[2] and err[3] <= 1e-11 * np.linalg.norm(A)


@pytest.mark.parametrize("p,tol", [(-1, 1e-3), (4, 1e-4)])
def test_ras_with_ilut_local_solvers(p, tol):
    dims = (6, 5, 4)
    _, B, Ao = system(dims, 2.0, 7)
    n = Ao.n
    r = I.test_vector(7, 3 * n)
    whole = O.ILU(Ao, ilut=(p, tol)).apply(r)
    assert np.array_equal(O.RAS(Ao, dims, (1, 1, 1), 0, ilut=(p, tol)).apply(r), whole)
    # singleton boxes: block Jacobi
    z = O.RAS(Ao, dims, dims, 0, ilut=(p, tol)).apply(r).reshape(-1, 3)
    ref = np.stack([np.linalg.solve(B[c, 3], r.reshape(-1, 3)[c]) for c in range(n)])
    assert np.allclose(z, ref, rtol=1e-12, atol=1e-14)


def test_ilut_beats_ilu0_on_the_literal_reading():
    cfg = I.preset("C1", seed=0)
    dims = (cfg.nx, cfg.ny, cfg.nz)
    Ao = O.BCSR.from_stencil(*dims, I.blocks(cfg))
    b = Ao.spmv(I.x_true(cfg))
    its0 = O.gmres(Ao, b, pc=O.ILU(Ao), m=30, tol=1e-8, maxit=3000)["its"]
    out = O.gmres(Ao, b, pc=O.ILU(Ao, ilut=(-1, 1e-3)), m=30, tol=1e-8, maxit=3000)
    assert out["rc"] == 0 and out["relres"] <= 1e-8 and out["its"] < its0 / 4


def test_errors():
    _, B, Ao = system((3, 3, 2), 2.0, 8)
    with pytest.raises(O.OracleError):
        O.ILU(Ao, ilut=(-1, -1.0))
    B2 = B.copy()
    B2[4, 3] = 0.0
    with pytest.raises(O.OracleError) as e:
        O.ILU(O.BCSR.from_stencil(3, 3, 2, B2), ilut=(-1, 1e300))
    assert e.value.rc == O.ERR_ZERO_PIVOT and e.value.bad_cell == 4
