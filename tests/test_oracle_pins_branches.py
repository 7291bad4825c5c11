"""Pins for the oracle branches that the value checks elsewhere do not reach:
Adam past its first step, FGMRES's rule that three consecutive fallbacks hand
the rest of a cycle to the fallback preconditioner, and BiCGSTAB's breakdown
exits.  Each pin is written from the method's definition (Kingma & Ba for
Adam; the fallback rule of the learned preconditioner; van der Vorst's
iteration for BiCGSTAB), not from the oracle's code, and each is chosen so
that a plausible slip in the oracle fails it (tests/test_oracle_mutations.py
plants those slips in a copy of the oracle and checks that the pins catch
them).  No GPU needed.
"""
import numpy as np
import pytest

from paper_1602_05901_amd import inputs as I
import oracle as O
from oracle import unet as U

from cases import breakdown_systems, two_cell_blocks


# ---------------------------------------------------------------- Adam (Kingma & Ba 2015, Algorithm 1)

B1, B2, EPS = 0.9, 0.999, 1e-8


def test_adam_constant_gradient_steps_2_and_3():
    """With the same gradient g at every step the bias-corrected moments are
    exactly g and g^2 at every t, so every step moves p by lr*g/(|g|+eps).
    A bias correction that drops its exponent (1-b instead of 1-b^t) still
    passes at t = 1 and fails here from t = 2 on."""
    g = I.uniform(31, 6, 40, -2.0, 2.0)
    p = I.uniform(32, 6, 40, -1.0, 1.0)
    m = np.zeros(40)
    v = np.zeros(40)
    lr = 1e-2
    for t in (1, 2, 3):
        want = p - lr * g / (np.abs(g) + EPS)
        p, m, v = U.adam(p, g, m, v, t, lr)
        assert np.max(np.abs(p - want)) <= 1e-14, t
        # raw moments in closed form: (1 - b^t) g and (1 - b^t) g^2
        assert np.allclose(m, (1 - B1 ** t) * g, rtol=1e-14, atol=0)
        assert np.allclose(v, (1 - B2 ** t) * g * g, rtol=1e-12, atol=0)   # 1 - b2^t cancels digits


def test_adam_three_different_gradients_closed_form():
    """Three steps with different gradients against the moments written out
    as sums: m_3 = (1-b1)(b1^2 g1 + b1 g2 + g3), v_3 likewise with squares,
    p_3 = p_2 - lr m_3/(1-b1^3) / (sqrt(v_3/(1-b2^3)) + eps)."""
    gs = [I.uniform(40 + k, 6, 25, -1.0, 1.0) for k in range(3)]
    p0 = I.uniform(44, 6, 25, -1.0, 1.0)
    lr = 3e-3
    p, m, v = p0.copy(), np.zeros(25), np.zeros(25)
    ps = []
    for t, g in enumerate(gs, start=1):
        p, m, v = U.adam(p, g, m, v, t, lr)
        ps.append(p)
    g1, g2, g3 = gs
    m1, v1 = (1 - B1) * g1, (1 - B2) * g1 ** 2
    m2 = (1 - B1) * (B1 * g1 + g2)
    v2 = (1 - B2) * (B2 * g1 ** 2 + g2 ** 2)
    m3 = (1 - B1) * (B1 ** 2 * g1 + B1 * g2 + g3)
    v3 = (1 - B2) * (B2 ** 2 * g1 ** 2 + B2 * g2 ** 2 + g3 ** 2)
    e1 = p0 - lr * (m1 / (1 - B1)) / (np.sqrt(v1 / (1 - B2)) + EPS)
    e2 = e1 - lr * (m2 / (1 - B1 ** 2)) / (np.sqrt(v2 / (1 - B2 ** 2)) + EPS)
    e3 = e2 - lr * (m3 / (1 - B1 ** 3)) / (np.sqrt(v3 / (1 - B2 ** 3)) + EPS)
    for got, want in zip(ps, (e1, e2, e3)):
        assert np.max(np.abs(got - want)) <= 1e-13
    assert np.allclose(m, m3, rtol=1e-13, atol=1e-16) and np.allclose(v, v3, rtol=1e-13, atol=1e-18)


# ---------------------------------------------------------------- FGMRES fallback rule

def _c1_small(seed=2):
    cfg = I.GenConfig(6, 5, 4, I.LNK_IID, 1.0, 0.0, 2.0, 0, 1e3, 1.0, seed)
    A = O.BCSR.from_stencil(cfg.nx, cfg.ny, cfg.nz, I.blocks(cfg))
    b = A.spmv(I.x_true(cfg))
    return A, b


def test_fgmres_three_rejections_hand_the_cycle_to_the_fallback():
    """A map that is always rejected (it returns zero, so the column adds
    nothing and the residual estimate does not drop) is tried on the first
    three columns of every cycle and then not again until the restart; every
    column falls back."""
    A, b = _c1_small()
    F = O.ILU(A)
    calls = []

    def net(v):
        calls.append(len(calls))
        return np.zeros_like(v)

    m = 5
    out = O.fgmres(A, b, pc=net, fallback=F, theta=0.99, m=m, tol=1e-10, maxit=200)
    assert out["rc"] == O.OK
    its, cycles = out["its"], out["restarts"]
    assert cycles >= 2 and its > 3 * cycles       # several cycles, each longer than three columns
    lengths = [m] * (cycles - 1) + [its - m * (cycles - 1)]
    assert 1 <= lengths[-1] <= m
    assert len(calls) == sum(min(3, n) for n in lengths)
    assert out["fallbacks"] == its
    # the solve itself is the fallback's GMRES
    g = O.gmres(A, b, pc=F, m=m, tol=1e-10, maxit=200)
    assert its == g["its"] and np.linalg.norm(out["x"] - g["x"]) <= 1e-9 * np.linalg.norm(g["x"])


def test_fgmres_acceptance_resets_the_consecutive_count():
    """Calls alternate reject, reject, accept (an accepted column is the
    fallback's own, exact ILU(0) apply, which reduces the estimate on this
    system): three rejections in a row never happen, so the map is called on
    every column, and exactly the rejected calls fall back."""
    A, b = _c1_small(seed=3)
    F = O.ILU(A)
    calls = []

    def net(v):
        k = len(calls)
        calls.append(k)
        return F.apply(v) if k % 3 == 2 else np.zeros_like(v)

    out = O.fgmres(A, b, pc=net, fallback=F, theta=0.99, m=30, tol=1e-10, maxit=200)
    assert out["rc"] == O.OK and out["its"] >= 4
    assert len(calls) == out["its"]
    assert out["fallbacks"] == sum(1 for k in calls if k % 3 != 2)


# ---------------------------------------------------------------- BiCGSTAB breakdown (van der Vorst 1992)

@pytest.mark.parametrize("case", ["rv0", "omega0"])
def test_bicgstab_breakdown_exits(case):
    name, A6, b, x_want = [c for c in breakdown_systems() if c[0] == case][0]
    assert abs(np.linalg.det(A6)) > 0.1                # the system itself is regular
    if case == "rv0":
        assert b @ (A6 @ b) == 0.0
    else:
        s = b - 4.0 * (A6 @ b)
        assert s[0] == 0.0 and np.linalg.norm(s) > 0 and (A6 @ s) @ s == 0.0
    A = O.BCSR.from_stencil(2, 1, 1, two_cell_blocks(A6))
    assert np.array_equal(A.spmv(b), A6 @ b)
    out = O.bicgstab(A, b, pc=None, tol=1e-12, maxit=50)
    assert out["rc"] == O.BREAKDOWN and out["its"] == (0 if case == "rv0" else 1)
    assert np.array_equal(out["x"], x_want)
    if case == "omega0":
        # omega = 0 ends the iteration that produced it, before the iteration
        # limit is looked at (after a first iteration r = s is orthogonal to
        # r^, so without that exit the next iteration's rho = 0 test would
        # report the same breakdown; with maxit = 1 it would not be reached)
        one = O.bicgstab(A, b, pc=None, tol=1e-12, maxit=1)
        assert one["rc"] == O.BREAKDOWN and np.array_equal(one["x"], x_want)
    # the reported residual is the recomputed one of the x handed back
    assert out["relres"] == pytest.approx(np.linalg.norm(b - A6 @ x_want) / np.linalg.norm(b), rel=1e-15)
    # a regular system that only BiCGSTAB's short recurrences fail on: GMRES solves it
    g = O.gmres(A, b, pc=None, m=30, tol=1e-12, maxit=50)
    assert g["rc"] == O.OK and np.allclose(A6 @ g["x"], b, atol=1e-11)
