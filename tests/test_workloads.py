"""Pins of the closed-form exact solutions used as references.

Each closed form is checked against the PDE it solves: a characteristic
integrated by scipy's adaptive ODE solver (library routine), or the PDE
residual by centred differences."""
import math

import numpy as np
from scipy.integrate import solve_ivp

import workloads as W


def test_c2_flow_map_matches_ode():
    xs = np.array([0.0, 0.3, 0.9, 1.0, 1.1, 1.7, 1.99])
    for t in (0.05, 0.4, 1.3, 2.5):
        sol = solve_ivp(lambda s, y: -(1 + 0.5 * np.sin(np.pi * y)), (0, t), xs, rtol=1e-12, atol=1e-13)
        foot = sol.y[:, -1]
        np.testing.assert_allclose(W.c2_exact(xs, None, t), W.c2_u0(foot), atol=1e-9)


def test_c2_exact_satisfies_advective_pde():
    x = np.linspace(0.05, 1.95, 37)
    t, h = 0.7, 1e-5
    ut = (W.c2_exact(x, None, t + h) - W.c2_exact(x, None, t - h)) / (2 * h)
    ux = (W.c2_exact(x + h, None, t) - W.c2_exact(x - h, None, t)) / (2 * h)
    res = ut + (1 + 0.5 * np.sin(np.pi * x)) * ux
    assert np.abs(res).max() < 1e-6


def test_c3_rotation_exact():
    x = np.array([0.2, 0.5, 0.7, 0.9])
    y = np.array([0.4, 0.5, 0.5, 0.1])
    t, h = 0.3, 1e-5
    ut = (W.c3_exact(x, y, t + h) - W.c3_exact(x, y, t - h)) / (2 * h)
    ux = (W.c3_exact(x + h, y, t) - W.c3_exact(x - h, y, t)) / (2 * h)
    uy = (W.c3_exact(x, y + h, t) - W.c3_exact(x, y - h, t)) / (2 * h)
    assert np.abs(ut - (y - 0.5) * ux + (x - 0.5) * uy).max() < 1e-6
    np.testing.assert_allclose(W.c3_exact(x, y, 2 * math.pi), W.c3_u0(x, y), atol=1e-12)


def test_x6_closed_form_solves_conservative_pde_and_matches_ic():
    """Section 5.2: phi_t + (-sin(x) phi)_x = 0 with the printed initial
    condition sin(2 atan(e^-1 tan(x/2))) / sin(x)."""
    x = np.linspace(0.1, 2 * math.pi - 0.1, 41)
    x = x[np.abs(x - math.pi) > 0.05]
    ic = np.sin(2 * np.arctan(math.exp(-1) * np.tan(x / 2))) / np.sin(x)
    np.testing.assert_allclose(W.x6_exact(x, None, 0.0), ic, rtol=1e-12)
    t, h = 0.4, 1e-5
    pt = (W.x6_exact(x, None, t + h) - W.x6_exact(x, None, t - h)) / (2 * h)
    flux = lambda xx: -np.sin(xx) * W.x6_exact(xx, None, t)
    fx = (flux(x + h) - flux(x - h)) / (2 * h)
    assert np.abs(pt + fx).max() < 1e-6
    # "dampens into a constant": phi == 1 at t = 1
    np.testing.assert_allclose(W.x6_exact(x, None, 1.0), 1.0, atol=1e-14)


def test_config_time_steps():
    """dt = 0.2 * min node gap * dx / max|a| for the three measured shapes."""
    assert abs(W.c1().dt - 1.6516e-3) < 5e-8
    assert abs(W.c2().dt - 8.118e-8) < 5e-11
    assert abs(W.c3().dt - 1.0323e-4) < 5e-9
    assert W.c1().dofs == 144 and W.c2().dofs == 1114112 and W.c3().dofs == 5308416
