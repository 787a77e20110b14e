"""Pins of the oracle's reference-element tables and building blocks.

Each check ties the oracle to something other than itself: numpy's library
quadrature rules, exact integrals of monomials, the interpolation property of
the Lagrange basis, scipy's barycentric interpolator, and the textbook order
conditions of explicit Runge-Kutta tableaux.
"""
import numpy as np
import pytest
from scipy.interpolate import BarycentricInterpolator


@pytest.mark.parametrize("n", list(range(1, 21)))
def test_gauss_legendre_matches_numpy(ora, n):
    xi, w = ora.nodes(0, n)
    t, wl = np.polynomial.legendre.leggauss(n)
    order = np.argsort((1 - t) / 2)
    np.testing.assert_allclose(xi, ((1 - t) / 2)[order], rtol=0, atol=2e-16)
    np.testing.assert_allclose(w, (wl / 2)[order], rtol=0, atol=2e-15)


@pytest.mark.parametrize("n", [1, 2, 5, 9, 13, 17])
def test_gauss_legendre_exact_to_degree_2n_minus_1(ora, n):
    xi, w = ora.nodes(0, n)
    for k in range(2 * n):
        assert abs(np.dot(w, xi ** k) - 1.0 / (k + 1)) < 1e-14
    # and not exact at degree 2n (the defect is visible in FP64 for small n)
    if n <= 5:
        assert abs(np.dot(w, xi ** (2 * n)) - 1.0 / (2 * n + 1)) > 1e-12


@pytest.mark.parametrize("n", list(range(1, 18)))
def test_chebyshev_gauss_nodes_closed_form(ora, n):
    """Section 3, eq. gaussquad (reading: n = N+1 points, angle (j+1/2) pi/n)."""
    xi, _ = ora.nodes(1, n)
    t, _ = np.polynomial.chebyshev.chebgauss(n)
    np.testing.assert_allclose(xi, np.sort((1 - t) / 2), atol=2e-16)


@pytest.mark.parametrize("n", [2, 5, 7, 8, 12])
def test_chebyshev_gauss_weights_interpolatory(ora, n):
    """Interpolatory weights: exact for every polynomial of degree < n."""
    xi, w = ora.nodes(1, n)
    for k in range(n):
        assert abs(np.dot(w, xi ** k) - 1.0 / (k + 1)) < 1e-14
    # equal to the integral of each Lagrange basis polynomial
    for j in range(n):
        e = np.zeros(n)
        e[j] = 1
        c = np.polynomial.polynomial.polyfit(xi, e, n - 1)
        ci = np.polynomial.polynomial.polyint(c)
        assert abs(np.polynomial.polynomial.polyval(1.0, ci) - w[j]) < 1e-8


def test_timestep_reading_matches_printed_dt(ora):
    """Section 5.2 prints dt = 1.97e-2 for H=4, P=6 on [0, 2 pi]: the gap
    between the element edge and the first Chebyshev-Gauss node with n = P+1
    points, times dx, over |u|max = 1 (reading of eq. 1d_delt_condition)."""
    import os
    path = os.path.join(os.path.dirname(__file__), "golden", "timestep.txt")
    printed = float([l.split()[1] for l in open(path) if l.startswith("x6_dt")][0])
    xi, _ = ora.nodes(1, 7)
    dt = xi[0] * (2 * np.pi / 4)
    assert float("%.2e" % dt) == printed
    # the literal "N nodes" reading does not reproduce it
    xi6, _ = ora.nodes(1, 6)
    assert float("%.2e" % (xi6[0] * np.pi / 2)) != printed


@pytest.mark.parametrize("family", [0, 1])
@pytest.mark.parametrize("n", [2, 5, 9, 17])
def test_lagrange_basis(ora, family, n):
    xi, _ = ora.nodes(family, n)
    for i in range(n):
        np.testing.assert_allclose(ora.lagrange(xi, xi[i]), np.eye(n)[i], atol=1e-13)
    rng = np.random.default_rng(1)
    f = rng.normal(size=n)
    interp = BarycentricInterpolator(xi, f)
    for t in rng.uniform(-0.05, 1.05, size=7):
        l = ora.lagrange(xi, t)
        assert abs(l.sum() - 1) < 1e-10
        assert abs(np.dot(l, f) - interp(t)) < 1e-9 * max(1, np.abs(f).max())


def _order_conditions(s, A, b, c):
    return {
        1: b[:s].sum() - 1,
        2: np.dot(b[:s], c[:s]) - 0.5,
        3: max(abs(np.dot(b[:s], c[:s] ** 2) - 1 / 3),
               abs(np.dot(b[:s], A[:s, :s] @ c[:s]) - 1 / 6)),
        4: max(abs(np.dot(b[:s], c[:s] ** 3) - 1 / 4),
               abs(np.dot(b[:s] * c[:s], A[:s, :s] @ c[:s]) - 1 / 8),
               abs(np.dot(b[:s], A[:s, :s] @ c[:s] ** 2) - 1 / 12),
               abs(np.dot(b[:s], A[:s, :s] @ A[:s, :s] @ c[:s]) - 1 / 24)),
    }


@pytest.mark.parametrize("rk,order", [(1, 1), (2, 2), (3, 3), (4, 4), (5, 2), (6, 3), (7, 2)])
def test_rk_tableau_order_conditions(ora, rk, order):
    s, A, b, c = ora.rk_tableau(rk)
    # consistency c_i = sum_j a_ij and explicit (strictly lower triangular)
    np.testing.assert_allclose(A[:s, :s].sum(1), c[:s], atol=1e-15)
    assert np.all(np.triu(A[:s, :s]) == 0)
    cond = _order_conditions(s, A, b, c)
    for p in range(1, order + 1):
        assert abs(cond[p]) < 1e-14, (p, cond[p])
    if order < 4:
        assert abs(cond[order + 1]) > 1e-6
