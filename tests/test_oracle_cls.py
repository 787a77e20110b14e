"""Pins of the oracle's constrained least-squares solves (paper section
"Least-squares solution of the constrained system", eq. matrix_a).

HARD is checked against the textbook least-squares-with-equality solution via
an SVD null-space basis (Golub & Van Loan, LSE problem), computed in 50-digit
mpmath for tiny sizes and with numpy's SVD for larger ones; SOFT against
numpy's least squares of the stacked system; the 2D boundary pseudo-inverse
against numpy.linalg.pinv and the rank the corner dependencies imply.
"""
import mpmath
import numpy as np
import pytest


def lse_mpmath(C, d, phihat):
    """min ||x - phihat|| s.t. C x = d: x = C^+ d + Z Z^T phihat, Z = null(C)."""
    mpmath.mp.dps = 50
    Cm = mpmath.matrix(C.tolist())
    U, S, V = mpmath.svd_r(Cm)  # C = U diag(S) V
    m, n = C.shape
    Vt = V.T
    # particular solution C^+ d
    x = mpmath.matrix(n, 1)
    for k in range(m):
        coef = sum(U[i, k] * d[i] for i in range(m)) / S[k]
        for j in range(n):
            x[j] += coef * V[k, j]
    # projection of phihat on the null space: phihat - V_r^T V_r phihat
    ph = mpmath.matrix(phihat.tolist())
    proj = mpmath.matrix(n, 1)
    for k in range(m):
        c = sum(V[k, j] * ph[j] for j in range(n))
        for j in range(n):
            proj[j] += c * V[k, j]
    out = x + ph - proj
    return np.array([float(out[j]) for j in range(n)])


@pytest.mark.parametrize("seed", range(6))
def test_hard_equals_lse_bruteforce(ora, seed):
    rng = np.random.default_rng(seed)
    n = int(rng.integers(4, 7))
    m = int(rng.integers(1, 5))
    C = rng.normal(size=(m, n))
    d = rng.normal(size=m)
    ph = rng.normal(size=n)
    x = ora.cls(C, d, ph, 0)
    ref = lse_mpmath(C, d, ph)
    np.testing.assert_allclose(x, ref, rtol=0, atol=1e-12)
    np.testing.assert_allclose(C @ x, d, atol=1e-12)


@pytest.mark.parametrize("seed", range(4))
def test_hard_is_a_projection(ora, seed):
    """HARD returns the nearest point of the affine set {C x = d}: solving
    again from that point changes nothing, and the correction is orthogonal
    to the null space of C (it lies in the row space)."""
    rng = np.random.default_rng(300 + seed)
    n, m = 17, 4
    C = rng.normal(size=(m, n))
    d = rng.normal(size=m)
    ph = rng.normal(size=n)
    x1 = ora.cls(C, d, ph, 0)
    x2 = ora.cls(C, d, x1, 0)
    np.testing.assert_allclose(x2, x1, rtol=0, atol=1e-13)
    _, _, Vt = np.linalg.svd(C)
    Z = Vt[m:].T  # null space basis
    np.testing.assert_allclose(Z.T @ (x1 - ph), 0.0, atol=1e-13)


@pytest.mark.parametrize("seed", range(4))
def test_hard_equals_lse_svd_larger(ora, seed):
    rng = np.random.default_rng(100 + seed)
    n, m = 17, 4
    C = rng.normal(size=(m, n))
    d = rng.normal(size=m)
    ph = rng.normal(size=n)
    U, S, Vt = np.linalg.svd(C)
    Z = Vt[m:].T
    ref = np.linalg.pinv(C) @ d + Z @ (Z.T @ ph)
    np.testing.assert_allclose(ora.cls(C, d, ph, 0), ref, atol=1e-12)


@pytest.mark.parametrize("seed", range(4))
def test_soft_equals_stacked_lstsq(ora, seed):
    """SOFT is the literal least-squares fit of the stacked system (eq.
    matrix_a): identity rows on phihat plus the constraint rows."""
    rng = np.random.default_rng(200 + seed)
    n = int(rng.integers(3, 12))
    m = int(rng.integers(1, 5))
    C = rng.normal(size=(m, n))
    d = rng.normal(size=m)
    ph = rng.normal(size=n)
    A = np.vstack([np.eye(n), C])
    rhs = np.concatenate([ph, d])
    ref = np.linalg.lstsq(A, rhs, rcond=None)[0]
    np.testing.assert_allclose(ora.cls(C, d, ph, 1), ref, atol=1e-12)


@pytest.mark.parametrize("family", [0, 1])
@pytest.mark.parametrize("n", [2, 3, 5, 9])
def test_boundary_pinv_2d(ora, family, n):
    """2D boundary rows (eq. 2dx_bnd_interpolate / 2dy_bnd_interpolate as
    constraints): rank 4n - 4 (one dependency per corner); the oracle's
    pseudo-inverse equals numpy's."""
    CB, CBp = ora.boundary_pinv(family, n)
    xi, _ = ora.nodes(family, n)
    l0, l1 = ora.lagrange(xi, 0.0), ora.lagrange(xi, 1.0)
    # row t of the left block evaluates the field at (0, eta_t)
    rng = np.random.default_rng(n)
    F = rng.normal(size=(n, n))  # F[j, i] = value at node (i, j)
    f = F.ravel()
    np.testing.assert_allclose(CB[:n] @ f, F @ l0, atol=1e-13)
    np.testing.assert_allclose(CB[n:2 * n] @ f, F @ l1, atol=1e-13)
    np.testing.assert_allclose(CB[2 * n:3 * n] @ f, l0 @ F, atol=1e-13)
    np.testing.assert_allclose(CB[3 * n:] @ f, l1 @ F, atol=1e-13)
    expect_rank = 4 * n - 4 if n >= 2 else 1
    assert np.linalg.matrix_rank(CB) == min(expect_rank, n * n)
    np.testing.assert_allclose(CBp, np.linalg.pinv(CB, rcond=1e-10), atol=1e-11)
