"""The algebra of the delayed second Gram-Schmidt pass (DCGS2), checked on the
CPU with numpy: the step the GPU path takes (one combined dot pass, then the
correction of the tentative vector and the projection of the new product,
norms from the Pythagorean identity, the Hessenberg column of the previous
step corrected afterwards) must give the Arnoldi process of classical
Gram-Schmidt applied twice: the same Hessenberg matrix to rounding, an
orthonormal basis, and A Q_k = Q_{k+1} H.  The GPU solver itself is held to
the oracle's GMRES by the GPU parity tests; this pins the derivation."""
import numpy as np
import pytest

LOST = 64.0 * np.finfo(np.float64).eps


def arnoldi_cgs2(A, q0, m):
    n = len(q0)
    Q = np.zeros((n, m + 1))
    H = np.zeros((m + 1, m))
    Q[:, 0] = q0 / np.linalg.norm(q0)
    for j in range(m):
        w = A @ Q[:, j]
        h1 = Q[:, :j + 1].T @ w
        w = w - Q[:, :j + 1] @ h1
        h2 = Q[:, :j + 1].T @ w
        w = w - Q[:, :j + 1] @ h2
        H[:j + 1, j] = h1 + h2
        H[j + 1, j] = np.linalg.norm(w)
        Q[:, j + 1] = w / H[j + 1, j]
    return Q, H


def arnoldi_dcgs2(A, q0, m, sloppy=0.0, seed=0):
    """Steps j = 0..m-1 as the GPU path runs them; column m-1 stays tentative
    (the cycle's last step keeps it).  sloppy > 0 spoils each tentative vector
    on purpose (a component sloppy * c along the basis and a norm off by a
    factor 1 + sloppy, its tentative column adjusted to match), so the
    corrections of the next step are exercised at O(sloppy) instead of O(eps)."""
    rng = np.random.default_rng(seed)
    n = len(q0)
    V = np.zeros((n, m + 1))
    H = np.zeros((m + 1, m))          # final (unrotated) columns
    V[:, 0] = q0 / np.linalg.norm(q0)
    ht, gam_prev = None, 0.0
    for j in range(m):
        K = j + 1
        w = A @ V[:, j]               # product of the tentative vector
        omega = w @ w                 # fused into the SpMV
        d = np.concatenate([V[:, :K].T @ V[:, j], V[:, :K].T @ w])   # one pass
        s, t = d[:j], d[K:K + j]
        alpha, tau = d[j], d[K + j]
        a = alpha - s @ s
        beta = 1.0 if (j == 0 or not a > 0) else np.sqrt(a)
        uj = (tau - s @ t) / beta
        d2 = omega - (t @ t + uj * uj)
        scale = 1.0 / np.sqrt(d2) if d2 > LOST * omega else 0.0
        q = (V[:, j] - V[:, :j] @ s) / beta          # delayed second pass on V_j
        if j > 0:
            V[:, j] = q
        V[:, j + 1] = (w - V[:, :j] @ t - uj * q) * scale
        c, f = sloppy * rng.standard_normal(K), 1.0 + sloppy
        if scale != 0.0:
            V[:, j + 1] = f * V[:, j + 1] + V[:, :K] @ c
        # host: finalise column j - 1, then the tentative column j
        if j >= 1:
            H[:j, j - 1] = ht[:j] + gam_prev * s
            H[j, j - 1] = gam_prev * beta
        u = np.concatenate([t, [uj]])
        ht = np.zeros(m + 1)
        ht[:K] = (u - H[:K, :j] @ s) / beta
        gam = np.sqrt(d2) / beta if d2 > LOST * omega else 0.0
        ht[K] = gam
        if scale != 0.0:
            ht[:K] -= gam * c / f
            ht[K] = gam / f
        gam_prev = ht[K]
    H[:, m - 1] = ht
    return V, H


def _system(n, seed, shift):
    rng = np.random.default_rng(seed)
    A = rng.standard_normal((n, n)) / np.sqrt(n) + shift * np.eye(n)
    return A, rng.standard_normal(n)


@pytest.mark.parametrize("seed,shift,m", [(0, 2.0, 12), (1, 0.5, 20), (2, 4.0, 30), (3, 1.0, 1)])
def test_dcgs2_equals_cgs2(seed, shift, m):
    A, b = _system(60, seed, shift)
    Qc, Hc = arnoldi_cgs2(A, b, m)
    Qd, Hd = arnoldi_dcgs2(A, b, m)
    nh = np.linalg.norm(Hc)
    # every column but the last (tentative) agrees to rounding; the last one
    # to the first pass's accuracy
    assert np.linalg.norm(Hd[:, :m - 1] - Hc[:, :m - 1]) <= 1e-12 * nh
    assert np.linalg.norm(Hd[:, m - 1] - Hc[:, m - 1]) <= 1e-10 * nh
    # the final basis vectors are the CGS2 ones and orthonormal
    Qf = Qd[:, :m]
    assert np.linalg.norm(Qf - Qc[:, :m]) <= 1e-12
    assert np.linalg.norm(np.eye(m) - Qf.T @ Qf) <= 1e-13
    # Arnoldi relation with the tentative last vector
    assert np.linalg.norm(A @ Qf - Qd @ Hd) <= 1e-12 * np.linalg.norm(A)


@pytest.mark.parametrize("seed,shift,m", [(5, 2.0, 12), (6, 0.7, 25)])
def test_dcgs2_corrections_with_spoiled_tentative_vectors(seed, shift, m):
    """Tentative vectors a thousandth off the orthonormal basis: the delayed
    pass must still give the CGS2 basis and Hessenberg columns (a wrong sign
    or term in a correction shows at O(1e-3))."""
    A, b = _system(60, seed, shift)
    Qc, Hc = arnoldi_cgs2(A, b, m)
    Qd, Hd = arnoldi_dcgs2(A, b, m, sloppy=1e-3, seed=seed)
    nh = np.linalg.norm(Hc)
    assert np.linalg.norm(Hd[:, :m - 1] - Hc[:, :m - 1]) <= 1e-10 * nh
    assert np.linalg.norm(Qd[:, :m] - Qc[:, :m]) <= 1e-10
    assert np.linalg.norm(A @ Qd[:, :m] - Qd @ Hd) <= 1e-12 * np.linalg.norm(A)
    # the last column is the spoiled tentative one
    assert np.linalg.norm(Hd[:, m - 1] - Hc[:, m - 1]) > 1e-6 * nh


def test_dcgs2_gmres_minimiser():
    """The least-squares solution over the DCGS2 Hessenberg matrix is the GMRES
    iterate: it minimises ||b - A x|| over the Krylov space (dense check)."""
    A, b = _system(50, 4, 1.5)
    m = 8
    V, H = arnoldi_dcgs2(A, b, m)
    e1 = np.zeros(m + 1)
    e1[0] = np.linalg.norm(b)
    y = np.linalg.lstsq(H, e1, rcond=None)[0]
    x = V[:, :m] @ y
    K = np.column_stack([np.linalg.matrix_power(A, k) @ b for k in range(m)])
    c = np.linalg.lstsq(A @ K, b, rcond=None)[0]
    x_ref = K @ c
    assert np.linalg.norm(x - x_ref) <= 1e-9 * np.linalg.norm(x_ref)
    assert abs(np.linalg.norm(b - A @ x) - np.linalg.norm(e1 - H @ y)) <= 1e-10 * np.linalg.norm(b)


def test_dcgs2_breakdown_when_the_space_is_invariant():
    """A = I: the second vector has no component left; d2 is rounding only, the
    next vector is zero and the subdiagonal entry is zero (breakdown)."""
    A = np.eye(10)
    b = np.arange(1.0, 11.0)
    V, H = arnoldi_dcgs2(A, b, 1)
    assert H[1, 0] == 0.0 and np.all(V[:, 1] == 0.0)
    assert abs(H[0, 0] - 1.0) <= 1e-15
