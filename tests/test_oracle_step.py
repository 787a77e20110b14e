"""Pins of the oracle's full step against properties the mathematics fixes.

* polynomial reproduction: with constant velocity and exact inflow ghost
  values, a polynomial of degree <= N is advected exactly (sections 4.1-4.3
  and the 2D scheme): the interpolant, the moved-point remap and the traces
  are all exact, and the exact field satisfies every constraint row;
* the 2D remap with constant velocity factorises (V = A (x) B), so a
  separable field steps like the outer product of two 1D steps;
* the mass targets integrate a flux cubic in t exactly with the tableau's
  quadrature (RK3, RK4);
* constants are preserved by any divergence-free nodal velocity;
* mirror symmetry x -> L - x, a -> -a;
* HARD mass rows make the global mass telescope (periodic);
* the constraint residuals and the energy row's fixed point;
* convergence to the closed-form solutions of the workloads;
* for a linear velocity, one step is the method's stability polynomial
  (closed form, every tableau, both forms, 1D and 2D);
* meshes periodic in one direction with ghost values on the sides of the
  other reproduce polynomials across the ghost sides and never read the
  ghost values of the periodic sides;
* zero velocity (every face on the tie rule) leaves a global polynomial
  unchanged.
"""
import math

import numpy as np
import pytest

import workloads as W


def _poly_workload(dim, n, deg, family=W.GL, rk=4, cmask=W.BOUNDARY, mode=W.HARD, vel=(0.7, -0.4)):
    rng = np.random.default_rng(deg + 10 * n)
    cx = rng.normal(size=deg + 1)
    cy = rng.normal(size=deg + 1)
    a, b = vel
    if dim == 1:
        f = lambda x, y, t: np.polynomial.polynomial.polyval(x - a * t, cx)
        wl = W.Workload(name="p1", dim=1, kx=5, ky=1, n=n, family=family, x0=-0.3, x1=1.2, y0=0, y1=1,
                        bc=W.GHOST, form=W.ADVECTIVE, rk=rk, cmask=cmask, mode=mode,
                        dt=0.2 * W.min_gap(family, n) * 0.3 / abs(a), nsteps=3,
                        u0=lambda x, y: f(x, y, 0.0), vel=lambda x, y: (a * np.ones_like(x), 0.0, 0.0),
                        exact=f)
    else:
        f = lambda x, y, t: (np.polynomial.polynomial.polyval(x - a * t, cx)
                             * np.polynomial.polynomial.polyval(y - b * t, cy))
        wl = W.Workload(name="p2", dim=2, kx=3, ky=2, n=n, family=family, x0=-0.3, x1=1.2, y0=0.1, y1=0.9,
                        bc=W.GHOST, form=W.ADVECTIVE, rk=rk, cmask=cmask, mode=mode,
                        dt=0.2 * W.min_gap(family, n) * 0.4 / max(abs(a), abs(b)), nsteps=2,
                        u0=lambda x, y: f(x, y, 0.0),
                        vel=lambda x, y: (a * np.ones_like(x), b * np.ones_like(x), 0.0),
                        exact=f)
    return wl


@pytest.mark.parametrize("mode", [W.HARD, W.SOFT])
@pytest.mark.parametrize("n,deg", [(4, 3), (6, 5), (9, 8), (9, 3)])
def test_polynomial_reproduction_1d(ora, n, deg, mode):
    w = _poly_workload(1, n, deg, mode=mode)
    phi, st = ora.run_workload(w)
    ex = w.exact_at(w.nsteps * w.dt)
    np.testing.assert_allclose(phi, ex, atol=1e-12 * max(1, np.abs(ex).max()))
    assert st.flags == 0


@pytest.mark.parametrize("rk", [2, 3, 4])
def test_polynomial_reproduction_1d_mass_energy(ora, rk):
    """Degree <= 1 polynomials: the face values are linear in t, so every
    tableau integrates the mass balance exactly; energy is quadratic in t so
    RK3/RK4 (Simpson) integrate it exactly and Heun does not."""
    w = _poly_workload(1, 6, 1, rk=rk, cmask=W.BOUNDARY | W.MASS | W.ENERGY)
    w.energy_tol = 0.0
    w.energy_maxit = 6
    phi, st = ora.run_workload(w)
    ex = w.exact_at(w.nsteps * w.dt)
    err = np.abs(phi - ex).max()
    if rk >= 3:
        assert err < 1e-12
    else:
        assert err < 1e-9  # Heun's trapezoid leaves an O(dt^3) energy defect
    assert st.resid_mass < 1e-13 and st.resid_energy < 1e-13
    # the stop is strict (|phi^(k) - phi^(k-1)| < tol), so tol = 0 always runs
    # the full count even when an exact fixed point is reached
    assert st.max_picard == 6


@pytest.mark.parametrize("mode", [W.HARD, W.SOFT])
@pytest.mark.parametrize("rk", [3, 4])
def test_mass_target_quadrature_exact_for_cubic_flux(ora, rk, mode):
    """A cubic moved at constant speed: the face values, and with them the
    mass fluxes, are cubic in t, which the tableau's own quadrature (Simpson's
    weights for Kutta's third order and for RK4) integrates exactly, while
    equal weights at the same abscissae would not.  After one step every
    element whose inflow face is interior is exact; the inflow element's
    stage values come from ghost rows that are linear in t."""
    w = _poly_workload(1, 6, 3, rk=rk, cmask=W.BOUNDARY | W.MASS, mode=mode)
    w.nsteps = 1
    phi, st = ora.run_workload(w)
    ex = w.exact_at(w.dt)
    err = np.abs((phi - ex).reshape(w.K, w.n))
    assert err[1:].max() < 1e-12 * max(1.0, np.abs(ex).max())
    assert st.flags == 0


@pytest.mark.parametrize("mode", [W.HARD, W.SOFT])
@pytest.mark.parametrize("n,deg", [(3, 2), (5, 4), (5, 2), (17, 16), (17, 9)])
def test_polynomial_reproduction_2d(ora, n, deg, mode):
    w = _poly_workload(2, n, deg, mode=mode)
    phi, st = ora.run_workload(w)
    ex = w.exact_at(w.nsteps * w.dt)
    np.testing.assert_allclose(phi, ex, atol=1e-11 * max(1, np.abs(ex).max()))


@pytest.mark.parametrize("n", [4, 6])
def test_2d_remap_factorises_for_constant_velocity(ora, n):
    """V = A (x) B for constant velocity: the unconstrained 2D step of
    f(x) g(y) is the outer product of the 1D steps of f and g."""
    kx, ky, a, b = 3, 2, 0.8, -0.5
    dt = 0.15 * W.min_gap(W.GL, n) * min(1.0 / kx, 1.0 / ky) / 0.8
    rng = np.random.default_rng(n)
    fx = rng.normal(size=(kx, n))
    gy = rng.normal(size=(ky, n))
    p1x = ora.params_from(_poly_workload(1, n, 1), kx=kx, x0=0.0, x1=1.0, bc=W.PERIODIC, cmask=0)
    p1y = ora.params_from(_poly_workload(1, n, 1), kx=ky, x0=0.0, x1=1.0, bc=W.PERIODIC, cmask=0)
    ox, _ = ora.step(p1x, fx.ravel(), a=np.full(kx * n, a), dt=dt)
    oy, _ = ora.step(p1y, gy.ravel(), a=np.full(ky * n, b), dt=dt)
    ox, oy = ox.reshape(kx, n), oy.reshape(ky, n)
    p2 = ora.params_from(_poly_workload(2, n, 1), kx=kx, ky=ky, x0=0.0, x1=1.0, y0=0.0, y1=1.0,
                         bc=W.PERIODIC, cmask=0)
    K = kx * ky
    f2 = np.zeros((K, n * n))
    ref = np.zeros((K, n * n))
    for e in range(K):
        ex, ey = e % kx, e // kx
        f2[e] = np.outer(gy[ey], fx[ex]).ravel()   # index jj*n + ii
        ref[e] = np.outer(oy[ey], ox[ex]).ravel()
    vel = np.concatenate([np.full(K * n * n, a), np.full(K * n * n, b)])
    o2, st = ora.step(p2, f2.ravel(), a=vel, dt=dt)
    np.testing.assert_allclose(o2.reshape(K, n * n), ref, atol=1e-12)


@pytest.mark.parametrize("dim", [1, 2])
def test_constant_preserved_divergence_free(ora, dim):
    if dim == 1:
        w = W.c1(n=7, K=6, nsteps=5)
    else:
        w = W.c3(kx=4, n=5, nsteps=3)
        w.bc = W.GHOST
    p = ora.params_from(w)
    a, _ = w.velocity()
    ghost = np.ones(ora.lib().ora_ghost_count(p)) if w.bc != W.PERIODIC else None
    phi, st = ora.step(p, np.ones(w.dofs), a=a, ghost=ghost, dt=w.dt, nsteps=w.nsteps)
    np.testing.assert_allclose(phi, 1.0, atol=1e-13)


def test_constant_preserved_boundary_only_variable_velocity(ora):
    w = W.c2(K=12, n=9, nsteps=4, cmask=W.BOUNDARY)
    p = ora.params_from(w)
    a, _ = w.velocity()
    phi, st = ora.step(p, np.ones(w.dofs), a=a, dt=w.dt, nsteps=w.nsteps)
    assert st.flags == 0
    np.testing.assert_allclose(phi, 1.0, atol=1e-13)


@pytest.mark.parametrize("cmask", [W.BOUNDARY, W.BOUNDARY | W.MASS, W.BOUNDARY | W.MASS | W.ENERGY])
@pytest.mark.parametrize("form", [W.ADVECTIVE, W.CONSERVATIVE])
def test_mirror_symmetry_1d(ora, cmask, form):
    """x -> L - x with a -> -a maps the step onto itself (left/right faces,
    upwinding, fluxes and traces swap roles)."""
    K, n = 6, 7
    rng = np.random.default_rng(3)
    x0, x1 = 0.0, 1.0
    xi = W.nodes(W.GL, n)
    x = x0 + (np.arange(K)[:, None] + xi[None, :]) / K
    phi = np.exp(np.sin(2 * np.pi * x) + 0.3 * np.cos(4 * np.pi * x))
    a = 0.6 + 0.3 * np.sin(2 * np.pi * x + 0.4)
    w = W.c1(n=n, K=K)
    p = ora.params_from(w, x0=x0, x1=x1, cmask=cmask, form=form, energy_tol=0.0, energy_maxit=5)
    dt = 0.2 * W.min_gap(W.GL, n) / K
    o1, s1 = ora.step(p, phi.ravel(), a=a.ravel(), dt=dt, nsteps=3)
    o2, s2 = ora.step(p, phi[::-1, ::-1].ravel(), a=-a[::-1, ::-1].ravel(), dt=dt, nsteps=3)
    np.testing.assert_allclose(o2.reshape(K, n)[::-1, ::-1], o1.reshape(K, n), atol=1e-12)
    assert s1.flags == 0


def test_mass_telescopes_with_hard_mass_row(ora):
    """With a HARD mass row and upwind face fluxes, the per-element mass
    updates (eq. remap_mass) telescope, so the global mass changes only by
    the volume term (zero for a conservative form)."""
    K, n = 8, 6
    xi, wq = ora.nodes(0, n)
    x = (np.arange(K)[:, None] + xi[None, :]) / K
    phi = 1.0 + 0.5 * np.sin(2 * np.pi * x)
    a = 0.8 + 0.3 * np.sin(2 * np.pi * x)
    w = W.c1(n=n, K=K)
    p = ora.params_from(w, x0=0.0, x1=1.0, cmask=W.BOUNDARY | W.MASS, form=W.CONSERVATIVE)
    dt = 0.2 * W.min_gap(W.GL, n) / K
    M0 = np.sum(phi * wq / K)
    out, st = ora.step(p, phi.ravel(), a=a.ravel(), dt=dt, nsteps=10)
    M1 = np.sum(out.reshape(K, n) * wq / K)
    assert abs(M1 - M0) < 1e-14
    assert st.resid_mass < 1e-14


def test_energy_picard_stops_and_holds_energy(ora):
    """Picard on the energy row (section "Local energy conservation"): with
    the paper's stop |phi^(k) - phi^(k-1)| < 1e-8 the iteration ends, the
    energy row then holds to well below that tolerance, and boundary and mass
    rows hold to round-off."""
    w = W.c2(K=16, n=9, nsteps=3)
    p = ora.params_from(w, energy_tol=1e-8, energy_maxit=60)
    a, _ = w.velocity()
    out, st = ora.step(p, w.initial(), a=a, dt=w.dt, nsteps=w.nsteps)
    assert st.flags == 0
    assert 1 <= st.max_picard < 60
    assert st.resid_energy < 1e-10 and st.resid_mass < 1e-14 and st.resid_boundary < 1e-12


def test_energy_sweeps_converge_hard(ora):
    """HARD energy row (C2 shape, tol = 0): the sweeps reach a fixed point,
    so 20, 21 and 22 sweeps give the same field to rounding."""
    w = W.c2(K=16, n=9, nsteps=1)
    a, _ = w.velocity()
    outs = []
    for it in (20, 21, 22):
        p = ora.params_from(w, energy_tol=0.0, energy_maxit=it)
        o, st = ora.step(p, w.initial(), a=a, dt=w.dt)
        outs.append(o)
    assert np.abs(outs[0] - outs[2]).max() < 1e-15
    assert np.abs(outs[0] - outs[1]).max() < 1e-15


def test_c1_converges_to_shifted_sine(ora):
    """Config-1 shape at full length: spectral accuracy against sin(pi(x-t))."""
    w = W.c1()
    phi, st = ora.run_workload(w)
    assert st.flags == 0
    err = w.l2_error(phi, w.nsteps * w.dt)
    assert err < 5e-8
    # a lower order on the same mesh is visibly less accurate (p-convergence)
    w5 = W.c1(n=5, nsteps=int(round(w.nsteps * w.dt / W.c1(n=5).dt)))
    phi5, _ = ora.run_workload(w5)
    assert w5.l2_error(phi5, w5.nsteps * w5.dt) > 100 * err


def test_c3_small_tracks_rotation(ora):
    w = W.c3(kx=8, n=7, nsteps=40)
    phi, st = ora.run_workload(w)
    assert st.flags == 0
    err = w.l2_error(phi, w.nsteps * w.dt)
    base = w.l2_error(w.initial(), w.nsteps * w.dt)
    assert err < 0.05 * base


def test_sampled_elements_match_full_step(ora):
    """The element mask computes the same values for the chosen elements."""
    w = W.c2(K=64, n=9, nsteps=1)
    p = ora.params_from(w, energy_tol=0.0, energy_maxit=4)
    a, _ = w.velocity()
    full, _ = ora.step(p, w.initial(), a=a, dt=w.dt)
    want = np.zeros(w.K, dtype=np.uint8)
    want[[0, 17, 63]] = 1
    part, _ = ora.step(p, w.initial(), a=a, dt=w.dt, want=want)
    for e in (0, 17, 63):
        np.testing.assert_array_equal(part.reshape(w.K, -1)[e], full.reshape(w.K, -1)[e])


@pytest.mark.parametrize("mode", [W.HARD, W.SOFT])
def test_linear_field_reproduction_2d_mass_energy(ora, mode):
    """2D counterpart of the 1D mass/energy exactness: a linear field moved by
    a constant velocity is linear in t at every fixed point, so its face
    fluxes are integrated exactly by RK4's Simpson weights (energy: quadratic
    in t) and the ghost values are exact under linear interpolation in t."""
    a, b = 0.7, -0.4
    f = lambda x, y, t: 0.3 + 0.7 * (x - a * t) - 0.4 * (y - b * t)
    n = 4
    w = W.Workload(name="lin2", dim=2, kx=3, ky=2, n=n, family=W.GL, x0=-0.3, x1=1.2, y0=0.1, y1=0.9,
                   bc=W.GHOST, form=W.ADVECTIVE, rk=4, cmask=W.BOUNDARY | W.MASS | W.ENERGY, mode=mode,
                   dt=0.2 * W.min_gap(W.GL, n) * 0.4 / 0.7, nsteps=3,
                   u0=lambda x, y: f(x, y, 0.0),
                   vel=lambda x, y: (a * np.ones_like(x), b * np.ones_like(x), 0.0), exact=f,
                   energy_tol=0.0, energy_maxit=6)
    phi, st = ora.run_workload(w)
    ex = w.exact_at(w.nsteps * w.dt)
    assert np.abs(phi - ex).max() < 1e-12
    assert st.resid_mass < 1e-13 and st.resid_energy < 1e-13


def test_divergence_from_interpolant_matches_exact_divergence_2d(ora):
    """D.a of the nodal velocity (dx != dy) equals the analytic divergence
    for a velocity field inside the interpolation space."""
    n, kx, ky = 5, 3, 2
    w = W.c3(kx=kx, ky=ky, n=n, nsteps=1)
    w.y1 = 0.5  # rectangular elements: dx = 1/3, dy = 1/4
    w.bc = W.PERIODIC
    w.cmask = W.BOUNDARY | W.MASS
    x, y = w.coords()
    u = 0.3 + 0.2 * x ** 2 - 0.1 * y
    v = -0.2 + 0.15 * y ** 3 + 0.05 * x
    div = 0.4 * x + 0.45 * y ** 2
    a = np.concatenate([u.ravel(), v.ravel()])
    p = ora.params_from(w, y1=0.5)
    phi0 = np.sin(2 * np.pi * x).ravel() + np.cos(4 * np.pi * y).ravel()
    dt = 0.2 * W.min_gap(W.GL, n) * (0.25 / 0.6)
    o1, s1 = ora.step(p, phi0, a=a, dt=dt, nsteps=2)
    o2, s2 = ora.step(p, phi0, a=a, div=div.ravel(), dt=dt, nsteps=2)
    np.testing.assert_allclose(o1, o2, atol=1e-12)


def test_conservative_energy_balance_tracks_exact_energy(ora):
    """Section 5.2 problem with all three constraints (SOFT, third order):
    the energy target follows the conservative balance law, whose volume term
    is -int(div a) phi^2, so the global energy ratio stays at 1."""
    w = W.x6(rk=3, cmask=W.BOUNDARY | W.MASS | W.ENERGY, mode=W.SOFT)
    phi, st = ora.run_workload(w)
    xi, wq = ora.nodes(w.family, w.n)
    x = w.x0 + (np.arange(w.K)[:, None] + xi[None, :]) * w.dx
    T = w.nsteps * w.dt
    ex = w.exact(x, None, T)
    P = phi.reshape(w.K, w.n)
    E = (P ** 2 * wq).sum() / (ex ** 2 * wq).sum()
    assert abs(E - 1.0) < 1e-3
    assert st.flags & ora.F_NOCONV == 0


def test_mass_telescopes_2d(ora):
    n, kx, ky = 4, 3, 3
    w = W.c3(kx=kx, ky=ky, n=n, nsteps=1)
    w.bc = W.PERIODIC
    x, y = w.coords()
    u = 0.5 + 0.2 * np.sin(2 * np.pi * y)
    v = -0.4 + 0.1 * np.cos(2 * np.pi * x)
    a = np.concatenate([u.ravel(), v.ravel()])
    p = ora.params_from(w, bc=W.PERIODIC, cmask=W.BOUNDARY | W.MASS, form=W.CONSERVATIVE)
    phi0 = (1.5 + np.sin(2 * np.pi * x) * np.cos(2 * np.pi * y)).ravel()
    Wq = w.quad_weights()
    dt = 0.2 * W.min_gap(W.GL, n) * (1 / kx) / 0.7
    out, st = ora.step(p, phi0, a=a, dt=dt, nsteps=4)
    assert abs(np.dot(Wq, out) - np.dot(Wq, phi0)) < 1e-14


@pytest.mark.parametrize("n,cmask,ok", [(2, W.BOUNDARY | W.MASS, False), (3, W.BOUNDARY | W.MASS, True),
                                        (3, W.BOUNDARY | W.MASS | W.ENERGY, False),
                                        (4, W.BOUNDARY | W.MASS | W.ENERGY, True)])
def test_2d_hard_rows_beyond_boundary_null_space_refused(ora, n, cmask, ok):
    """C_B has rank 4n-4, so null(C_B) has dimension (n-2)^2: HARD accepts
    at most that many mass/energy rows after the boundary block; SOFT (the
    stacked least squares) accepts any."""
    w = W.c3(kx=2, ky=2, n=n, nsteps=1)
    a, _ = w.velocity()
    g = w.ghost_rows(0.0, 1)
    for mode, expect in ((W.HARD, ok), (W.SOFT, True)):
        p = ora.params_from(w, cmask=cmask, mode=mode)
        if expect:
            out, st = ora.step(p, w.initial(), a=a, ghost=g, dt=w.dt, nsteps=1)
            assert np.all(np.isfinite(out))
        else:
            with pytest.raises(ValueError):
                ora.step(p, w.initial(), a=a, ghost=g, dt=w.dt, nsteps=1)


@pytest.mark.parametrize("form", [W.ADVECTIVE, W.CONSERVATIVE])
@pytest.mark.parametrize("rk", [1, 2, 3, 4])
@pytest.mark.parametrize("dim", [1, 2])
def test_linear_velocity_step_is_the_stability_polynomial(ora, dim, rk, form):
    """a = c x: one step gives u0 / R(c dt) (advective) or R(-d c dt) /
    R(c dt) u0 (conservative), R the degree-rk Taylor polynomial of e^z
    (tests/_linear_flow.py).  The same field with the next-order polynomial
    differs by more than 1e-10 here, so a dropped stage, a wrong weight or a
    wrong sign in the motion or in the source term fails."""
    import _linear_flow as LF
    w, a, div, ghost, expect = LF.case(dim, rk, form)
    p = ora.params_from(w)
    out, st = ora.step(p, w.initial(), a=a, div=div, ghost=ghost, dt=w.dt, nsteps=1)
    assert st.flags == 0
    np.testing.assert_allclose(out, expect, rtol=0, atol=4e-15)
    z = 0.9 * w.dt
    nxt = LF.stability(z, rk + 1)
    alt = w.initial() / nxt if form == W.ADVECTIVE else LF.stability(-dim * z, rk + 1) / nxt * w.initial()
    assert np.abs(alt - expect).max() > 1e-10


@pytest.mark.parametrize("mode", [W.HARD, W.SOFT])
@pytest.mark.parametrize("bc", [W.PERIODIC_X, W.PERIODIC_Y])
@pytest.mark.parametrize("deg,cmask", [(4, W.BOUNDARY), (1, W.BOUNDARY | W.MASS | W.ENERGY)])
def test_periodic_in_one_direction(ora, bc, deg, cmask, mode):
    """Periodic in x with ghost values on the bottom and top sides, or the
    other way round (tests/_onedir.py): a polynomial across the ghost sides,
    constant along the periodic direction, is advected exactly by a constant
    velocity (degree <= N with boundary rows; degree 1 with mass and energy
    rows, whose RK4 flux quadrature is then exact), with inflow from the
    exact solution.  The periodic sides' ghost values are NaN: reading one
    makes the field non-finite, and wrapping a ghost side brings in the
    opposite side's values instead of the inflow."""
    import _onedir
    w, g = _onedir.case(bc, deg, cmask, mode)
    a, _ = w.velocity()
    phi, st = ora.step(ora.params_from(w), w.initial(), a=a, ghost=g, dt=w.dt, nsteps=w.nsteps)
    ex = w.exact_at(w.nsteps * w.dt)
    assert np.all(np.isfinite(phi)) and st.flags == 0
    np.testing.assert_allclose(phi, ex, rtol=0, atol=1e-12 * max(1.0, np.abs(ex).max()))


@pytest.mark.parametrize("mode", [W.HARD, W.SOFT])
@pytest.mark.parametrize("cmask", [W.BOUNDARY, W.BOUNDARY | W.MASS | W.ENERGY])
@pytest.mark.parametrize("dim", [1, 2])
def test_zero_velocity_leaves_polynomials(ora, dim, cmask, mode):
    """a = 0 (tests/_zerovel.py): no particle moves and every face speed is
    zero, so each face takes the mean of its two traces.  A global polynomial
    of degree <= N has equal traces on both sides of every face (the ghost
    rows hold its own values), so three steps return it unchanged."""
    import _zerovel
    w = _zerovel.polynomial_case(dim, cmask, mode)
    phi, st = ora.run_workload(w)
    assert st.flags == 0
    np.testing.assert_allclose(phi, w.initial(), rtol=0, atol=1e-13)
