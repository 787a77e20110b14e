"""Pins of the oracle's backtracking interface values (eq. 4.11, section 4.3).

The element's edge value at t^{n+1} is phi^n at the foot of the
characteristic traced back over dt from the edge (times the source factor
in the conservative form), instead of the remapped polynomial at the edge
(eq. remap_bnd).  Pins:
  - constant velocity: the particles move exactly, the polynomial through
    the moved points is the translated element polynomial, so both interface
    values are the same number phi^n(xi_b - u dt) and whole runs agree to
    rounding (1D and 2D);
  - the paper's comparison (Fig. fig:bc, "no distinguishable result"),
    carried to the variable-velocity conservative problem of section 5.2:
    the L2 errors of the two variants agree within 10% for P = 4..7, while
    a dropped source factor, a forward trace or a half-length trace moves
    the backtracking error by factors of 20 and more.
"""
import numpy as np
import pytest

import workloads as W


def _paper_l2(ora, w, phi, t):
    xi, wq = ora.nodes(w.family, w.n)
    x = w.x0 + (np.arange(w.K)[:, None] + xi[None, :]) * w.dx
    ex = w.exact(x, None, t)
    return np.sqrt(((phi.reshape(w.K, w.n) - ex) ** 2 * wq * w.dx).sum(1)).sum()


@pytest.mark.parametrize("rk", [1, 4])
def test_backtrack_equals_interp_constant_velocity_1d(ora, rk):
    w = W.x1(P=5, H=4, rk=rk, T=0.5)
    a, sa = ora.run_workload(w)
    b, sb = ora.run_workload(w, iface=1)
    assert sa.flags == 0 and sb.flags == 0
    assert np.abs(a - b).max() <= 1e-13


def test_backtrack_equals_interp_constant_velocity_2d(ora):
    w = W.x9(P=4, H=3, rk=4, T=0.2)
    a, sa = ora.run_workload(w)
    b, sb = ora.run_workload(w, iface=1)
    assert sa.flags == 0 and sb.flags == 0
    assert np.abs(a - b).max() <= 1e-13


@pytest.mark.parametrize("P", [4, 5, 6, 7])
def test_backtrack_and_interp_equally_accurate_variable_velocity(ora, P):
    w = W.x6(P=P, H=4, rk=4)
    t = w.nsteps * w.dt
    a, _ = ora.run_workload(w)
    b, _ = ora.run_workload(w, iface=1)
    ea, eb = _paper_l2(ora, w, a, t), _paper_l2(ora, w, b, t)
    assert 0.9 <= eb / ea <= 1.1, (ea, eb)
    # the variants differ (the option is not ignored) by less than the error
    assert 0 < np.abs(a - b).max() < ea


def test_mixed_order_driver_refuses_backtracking(ora):
    wm = W.c4(kx=4, nsteps=1)
    p = ora.Params(dim=2, kx=wm.kx, ky=wm.ky, n=5, family=W.GL, bc=W.PERIODIC, form=W.ADVECTIVE, rk=4,
                   cmask=W.BOUNDARY, mode=W.HARD, energy_maxit=0, vel_kind=0, x0=0.0, x1=1.0, y0=0.0,
                   y1=1.0, energy_tol=0.0, iface=1)
    with pytest.raises(ValueError):
        ora.step_mixed(p, wm.orders, wm.initial(), a=wm.velocity(), dt=wm.dt, nsteps=1)
    p.iface = 0
    ora.step_mixed(p, wm.orders, wm.initial(), a=wm.velocity(), dt=wm.dt, nsteps=1)
