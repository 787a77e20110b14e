"""Pins of the oracle's HARD energy row (paper section "Local energy
conservation", eq. remap_energy, and the constrained least squares of eq.
matrix_a).

The paper linearises the energy row as sum W phi^(k-1) phi^(k) = E and
iterates.  A fixed point of that map is a point of the constraint set
{linear rows, sum W phi^2 = E} at which the distance to phihat is stationary
(the KKT point of the quadratic row).  Under HARD the map itself is
2-periodic, so the oracle reaches its fixed point by Newton's linearisation
of the same row.  These tests pin the result, not the route:

* against a 50-digit mpmath solve of the KKT system (null-space
  parametrisation and the secular equation of the multiplier), on random
  systems and on element-shaped ones (Gauss-Legendre weights, boundary and
  mass rows, a nearly constant field, where the energy row is nearly
  parallel to the mass row);
* the result is a fixed point of the paper's own map: one paper sweep from
  it changes nothing;
* the first Newton sweep lands, to first order, at the midpoint of the
  paper's 2-cycle;
* the stop rule and the flags (converged, not converged, no correction
  possible);
* in the full step: Newton sweeps settle (more sweeps change nothing), the
  energy row costs no accuracy on a C2-shaped mesh where the old
  2-periodic reading lost three orders of magnitude, and a constant field
  stays constant under boundary, mass and energy rows with a divergent
  velocity.
"""
import mpmath
import numpy as np
import pytest

import workloads as W


def _mp_null_lse(C, d, phihat):
    """phi1 = argmin ||phi - phihat|| s.t. C phi = d, and an orthonormal
    null-space basis Z of C, in mpmath (SVD)."""
    m, n = C.shape
    Cm = mpmath.matrix(C.tolist())
    U, S, V = mpmath.svd_r(Cm, full_matrices=True)
    x = mpmath.matrix(n, 1)
    for k in range(m):
        coef = sum(U[i, k] * mpmath.mpf(d[i]) for i in range(m)) / S[k]
        for j in range(n):
            x[j] += coef * V[k, j]
    ph = mpmath.matrix([mpmath.mpf(v) for v in phihat])
    for k in range(m):
        c = sum(V[k, j] * ph[j] for j in range(n))
        for j in range(n):
            ph[j] -= c * V[k, j]
    phi1 = x + ph
    Z = mpmath.matrix(n, n - m)
    for j in range(n):
        for k in range(n - m):
            Z[j, k] = V[m + k, j]
    return phi1, Z


def kkt_mpmath(C, d, Wq, s, T, phihat, dps=50):
    """min ||phi - phihat|| s.t. C phi = d, sum Wq (phi - s)^2 = T.

    phi = phi1 + Z alpha with ||phi - phihat||^2 = ||phi1 - phihat||^2 +
    |alpha|^2; stationarity gives alpha(nu) = -nu (I + nu Z^T D Z)^-1 Z^T D b
    (b = phi1 - s, D = diag(Wq)), and nu solves the secular equation
    (b + Z alpha)^T D (b + Z alpha) = T; the root nearest zero (started from
    its first-order estimate) is the nearest constrained point."""
    mpmath.mp.dps = dps
    C = np.atleast_2d(C)
    phi1, Z = _mp_null_lse(C, d, phihat)
    n, r = Z.rows, Z.cols
    D = [mpmath.mpf(v) for v in Wq]
    b = mpmath.matrix([phi1[j] - mpmath.mpf(s) for j in range(n)])
    ZDZ = mpmath.matrix(r, r)
    for a in range(r):
        for c in range(r):
            ZDZ[a, c] = sum(Z[j, a] * D[j] * Z[j, c] for j in range(n))
    ZDb = mpmath.matrix([sum(Z[j, a] * D[j] * b[j] for j in range(n)) for a in range(r)])
    Tm = mpmath.mpf(T)

    def alpha(nu):
        return mpmath.lu_solve(mpmath.eye(r) + nu * ZDZ, -nu * ZDb)

    def f(nu):
        al = alpha(nu)
        v = b + Z * al
        return sum(D[j] * v[j] ** 2 for j in range(n)) - Tm

    g0 = sum(D[j] * b[j] ** 2 for j in range(n)) - Tm
    nu0 = g0 / (2 * sum(x ** 2 for x in ZDb))
    nu = mpmath.findroot(f, nu0)
    phi = b + Z * alpha(nu)
    return np.array([float(phi[j] + mpmath.mpf(s)) for j in range(n)])


def _lse(C, d, phihat):
    """float LSE reference (numpy): nearest point of {C x = d}."""
    Cp = np.linalg.pinv(C)
    return phihat + Cp @ (d - C @ phihat)


def _random_case(seed, rel):
    rng = np.random.default_rng(seed)
    n = int(rng.integers(5, 9))
    m = int(rng.integers(1, 4))
    C = rng.normal(size=(m, n))
    d = rng.normal(size=m)
    ph = rng.normal(size=n)
    Wq = rng.uniform(0.5, 1.5, size=n)
    s = 0.1 * rng.normal()
    phi1 = _lse(C, d, ph)
    T = float(np.dot(Wq, (phi1 - s) ** 2)) * (1.0 + rel * rng.uniform(-1, 1))
    return C, d, Wq, s, T, ph


def _element_case(ora, seed, n=6, dx=1e-3, amp=1e-7, rel=1e-3):
    """An element of the method: Gauss-Legendre nodes, rows l(0), l(1) and the
    mass row W = dx w, a nearly constant field (variation amp) and a
    deviation energy target off by rel."""
    rng = np.random.default_rng(seed)
    xi, w = ora.nodes(W.GL, n)
    l0, l1 = ora.lagrange(xi, 0.0), ora.lagrange(xi, 1.0)
    Wq = dx * w
    ph = 1.0 + amp * rng.normal(size=n)
    C = np.vstack([l0, l1, Wq])
    d = np.array([l0 @ ph + 0.1 * amp * rng.normal(), l1 @ ph + 0.1 * amp * rng.normal(),
                  Wq @ ph * (1 + 0.1 * amp * rng.normal())])
    s = float(Wq @ ph / Wq.sum())
    phi1 = _lse(C, d, ph)
    T = float(np.dot(Wq, (phi1 - s) ** 2)) * (1.0 + rel * rng.uniform(-1, 1))
    return C, d, Wq, s, T, ph


@pytest.mark.parametrize("seed", range(6))
def test_energy_hard_equals_kkt_mpmath(ora, seed):
    C, d, Wq, s, T, ph = _random_case(seed, 0.05)
    x, k, fl = ora.energy_hard(C, d, Wq, s, T, ph, tol=0.0, maxit=30)
    ref = kkt_mpmath(C, d, Wq, s, T, ph)
    assert fl == 0
    np.testing.assert_allclose(x, ref, rtol=0, atol=1e-13)
    assert abs(np.dot(Wq, (x - s) ** 2) - T) < 1e-13 * T
    np.testing.assert_allclose(C @ x, d, atol=1e-13)


@pytest.mark.parametrize("seed", range(4))
def test_energy_hard_element_shaped_is_accurate(ora, seed):
    """Nearly constant element (the energy row and the mass row are nearly
    parallel, conditioning ~1e7): the deviation form keeps the result to a
    few ulps of the field, where the paper's phi^2 row loses ~eps * 1e7."""
    C, d, Wq, s, T, ph = _element_case(ora, seed)
    x, k, fl = ora.energy_hard(C, d, Wq, s, T, ph, tol=0.0, maxit=10)
    ref = kkt_mpmath(C, d, Wq, s, T, ph)
    assert fl == 0
    np.testing.assert_allclose(x, ref, rtol=0, atol=2e-15)
    # the correction is resolved: it moves the field by far more than that
    assert np.abs(ref - _lse(C, d, ph)).max() > 1e-12


def _paper_sweep(ora, C, d, Wq, s, T, ph, lin):
    """One sweep of the paper's map: nearest point to phihat with the linear
    rows and the row sum Wq lin phi = E, E = T + 2 s (Wq.phi) - s^2 sum Wq
    written for phi (the mass row, last in C, fixes Wq.phi = d[-1])."""
    E = T + 2.0 * s * d[-1] - s * s * Wq.sum()
    Ce = np.vstack([C, Wq * lin])
    return ora.cls(Ce, np.append(d, E), ph, 0)


@pytest.mark.parametrize("seed", range(4))
def test_result_is_a_fixed_point_of_the_papers_map(ora, seed):
    C, d, Wq, s, T, ph = _random_case(100 + seed, 0.05)
    C[-1] = Wq  # the last linear row is the mass row
    d[-1] = float(Wq @ _lse(C[:-1], d[:-1], ph)) if C.shape[0] > 1 else float(Wq @ ph)
    phi1 = _lse(C, d, ph)
    T = float(np.dot(Wq, (phi1 - s) ** 2)) * 1.03
    x, k, fl = ora.energy_hard(C, d, Wq, s, T, ph, tol=0.0, maxit=30)
    again = _paper_sweep(ora, C, d, Wq, s, T, ph, x)
    np.testing.assert_allclose(again, x, rtol=0, atol=1e-13)
    # ... while the paper's map does move the solution without the energy row
    assert np.abs(_paper_sweep(ora, C, d, Wq, s, T, ph, phi1) - phi1).max() > 1e-4


def test_first_sweep_is_the_midpoint_of_the_papers_two_cycle(ora):
    """From phi1 the paper's map jumps to phi2 and back (a 2-cycle); Newton's
    first sweep lands at (phi1 + phi2) / 2 up to second order in the
    correction."""
    C, d, Wq, s, T, ph = _random_case(7, 0.0)
    C[-1] = Wq
    phi1 = _lse(C, d, ph)
    T = float(np.dot(Wq, (phi1 - s) ** 2)) * (1 + 1e-4)
    phi2 = _paper_sweep(ora, C, d, Wq, s, T, ph, phi1)
    back = _paper_sweep(ora, C, d, Wq, s, T, ph, phi2)
    jump = np.abs(phi2 - phi1).max()
    assert np.abs(back - phi1).max() < 1e-3 * jump  # the cycle
    x1, _, _ = ora.energy_hard(C, d, Wq, s, T, ph, tol=0.0, maxit=1)
    assert np.abs(x1 - 0.5 * (phi1 + phi2)).max() < 1e-3 * jump


def test_stop_rule_counts_sweeps(ora):
    """Stop after the first sweep k whose change is below tol (strict); the
    outputs of maxit = 0, 1, 2, ... are the iterates."""
    C, d, Wq, s, T, ph = _random_case(3, 0.3)
    tol = 1e-12
    x, k, fl = ora.energy_hard(C, d, Wq, s, T, ph, tol=tol, maxit=40)
    assert fl == 0 and 2 <= k < 40
    its = [ora.energy_hard(C, d, Wq, s, T, ph, tol=0.0, maxit=j)[0] for j in range(0, k + 1)]
    steps = [np.abs(its[j] - its[j - 1]).max() for j in range(1, k + 1)]
    assert all(sj >= tol for sj in steps[:-1]) and steps[-1] < tol
    np.testing.assert_array_equal(x, its[k])


def test_flags_noconv_and_singular(ora):
    C, d, Wq, s, T, ph = _random_case(5, 0.05)
    # no real point has sum W (phi - s)^2 < 0: the sweeps never settle
    x, k, fl = ora.energy_hard(C, d, Wq, s, -1.0, ph, tol=1e-10, maxit=25)
    assert fl & ora.F_NOCONV and k == 25
    x, k, fl = ora.energy_hard(C, d, Wq, s, -1.0, ph, tol=0.0, maxit=25)
    assert not fl & ora.F_NOCONV  # tol = 0 runs a fixed count and flags nothing
    # a field equal to s (no linear rows, so phi1 = phihat exactly): the
    # linearised row is zero, no correction exists, and the energy is off
    ph0 = np.full(len(ph), s)
    none = np.zeros((0, len(ph)))
    x, k, fl = ora.energy_hard(none, np.zeros(0), Wq, s, 0.5, ph0, tol=1e-10, maxit=5)
    assert fl & ora.F_SINGULAR
    np.testing.assert_array_equal(x, ph0)
    # ... while with the energy already met there is nothing to flag
    x, k, fl = ora.energy_hard(none, np.zeros(0), Wq, s, 0.0, ph0, tol=1e-10, maxit=5)
    assert fl == 0 and k == 1


def test_step_newton_sweeps_settle(ora):
    """In the full step (C2 shape, boundary + mass + energy, HARD) further
    sweeps change nothing: the iteration has a fixed point, where the paper's
    linearisation alternated between two fields."""
    w = W.c2(K=64, n=9, nsteps=1)
    a, _ = w.velocity()
    outs = {}
    for it in (1, 2, 3, 8, 9):
        p = ora.params_from(w, energy_tol=0.0, energy_maxit=it)
        outs[it], st = ora.step(p, w.initial(), a=a, dt=w.dt)
        assert st.flags == 0
    # from the second sweep on the iterates agree to rounding (a converged
    # sweep can move a value by one ulp and back)
    for it in (2, 3, 8):
        np.testing.assert_allclose(outs[it], outs[9], rtol=0, atol=1e-15)
    assert np.abs(outs[1] - outs[9]).max() < 1e-12


def test_energy_row_costs_no_accuracy_on_a_fine_mesh(ora):
    """C2 shape (K = 2048, order 16, 5 steps, the paper's stop 1e-8): with the
    energy row the error against the closed form stays within 5% of the
    boundary + mass result, and every element converges.  Under the phi^2
    form of the target with the 2-periodic map, the same run was 300 times
    worse (rounding of the divergence defect, amplified by the near-parallel
    rows)."""
    res = {}
    for cm in (W.BOUNDARY | W.MASS, W.BOUNDARY | W.MASS | W.ENERGY):
        w = W.c2(K=2048, nsteps=5, cmask=cm)
        p = ora.params_from(w, energy_tol=1e-8, energy_maxit=50)
        a, _ = w.velocity()
        o, st = ora.step(p, w.initial(), a=a, dt=w.dt, nsteps=w.nsteps)
        assert st.flags == 0
        res[cm] = w.l2_error(o, w.nsteps * w.dt)
    lm, le = res[W.BOUNDARY | W.MASS], res[W.BOUNDARY | W.MASS | W.ENERGY]
    assert abs(le - lm) < 0.05 * lm, (lm, le)


@pytest.mark.parametrize("form", [W.ADVECTIVE])
def test_constant_field_kept_with_energy_rows(ora, form):
    """phi = const is a solution of the advective equation for any velocity;
    with a divergent velocity, boundary, mass and energy rows keep it (the
    deviation energy target is zero, and the mass target moves only by the
    rounding of the divergence defect)."""
    w = W.c2(K=32, n=9, nsteps=3)
    w.form = form
    x, _ = w.coords()
    a, _ = w.velocity()
    phi0 = np.full(x.size, 0.75)
    p = ora.params_from(w, cmask=W.BOUNDARY | W.MASS | W.ENERGY, energy_tol=1e-8, energy_maxit=50)
    o, st = ora.step(p, phi0, a=a, dt=w.dt, nsteps=w.nsteps)
    assert np.abs(o - 0.75).max() < 1e-13
    assert st.flags == 0
