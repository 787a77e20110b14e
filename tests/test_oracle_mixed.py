"""Pins of the oracle's mixed-order 2D step (orders per element; periodic,
boundary rows).  Independent checks: with one order everywhere it is the
uniform step (whose own pins hold); constants are preserved under a
divergence-free flow; translation of a smooth periodic field is as accurate
as the lowest order present allows; face coupling is symmetric under the
mirror map of the mesh."""
import math

import numpy as np
import pytest

import oracle
import workloads as W


def _params(kx, ky, n, mode=W.HARD, form=W.ADVECTIVE, rk=4):
    return oracle.Params(dim=2, kx=kx, ky=ky, n=n, family=W.GL, bc=W.PERIODIC, form=form, rk=rk,
                         cmask=W.BOUNDARY, mode=mode, energy_maxit=0, vel_kind=0, x0=0.0, x1=1.0, y0=0.0,
                         y1=1.0, energy_tol=0.0)


def _mixed(kx, ky, orders, u0, vel, dt):
    return W.MixedWorkload(name="t", kx=kx, ky=ky, orders=np.asarray(orders, dtype=np.int32), family=W.GL, dt=dt,
                           nsteps=1, u0=u0, vel=vel)


@pytest.mark.parametrize("mode", [W.HARD, W.SOFT])
@pytest.mark.parametrize("form", [W.ADVECTIVE, W.CONSERVATIVE])
def test_uniform_orders_equal_the_uniform_step(mode, form):
    kx, ky, n = 4, 3, 6
    rng = np.random.default_rng(1)
    ph = rng.uniform(0, 2 * math.pi, 3)
    vel = lambda x, y: (0.4 + 0.2 * np.sin(2 * math.pi * y + ph[0]), -0.3 + 0.1 * np.cos(2 * math.pi * x + ph[1]))
    u0 = lambda x, y: np.sin(2 * math.pi * x + ph[2]) * np.cos(2 * math.pi * y)
    dt = 0.2 * W.min_gap(W.GL, n) / max(kx, ky) / 0.6
    wm = _mixed(kx, ky, [n] * (kx * ky), u0, vel, dt)
    p = _params(kx, ky, n, mode, form)
    a = wm.velocity()
    g, st = oracle.step_mixed(p, wm.orders, wm.initial(), a=a, dt=dt, nsteps=2)
    # the uniform step on the same nodal data (its layout is the same when
    # every element has n^2 values)
    o, ost = oracle.step(p, wm.initial(), a=a, dt=dt, nsteps=2)
    assert np.max(np.abs(g - o)) <= 1e-13 * max(1.0, np.max(np.abs(o)))
    assert abs(st.resid_boundary - ost.resid_boundary) <= 1e-12


@pytest.mark.parametrize("mode", [W.HARD, W.SOFT])
def test_constant_preserved_with_mixed_orders(mode):
    kx = ky = 5
    rng = np.random.default_rng(2)
    orders = rng.choice([5, 7, 9, 13], size=kx * ky)
    wm = _mixed(kx, ky, orders, lambda x, y: 0 * x + 1.75, W.swirl_velocity, 0.2 * W.min_gap(W.GL, 13) / kx)
    p = _params(kx, ky, 5, mode)
    g, st = oracle.step_mixed(p, wm.orders, wm.initial(), a=wm.velocity(), dt=wm.dt, nsteps=3)
    assert np.max(np.abs(g - 1.75)) <= 1e-13


def _translation_error(orders, kx, nsteps=5):
    c = (0.3, -0.2)
    u0 = lambda x, y: np.sin(2 * math.pi * (x + 2 * y))
    wm = _mixed(kx, kx, orders, u0, lambda x, y: (0 * x + c[0], 0 * x + c[1]),
                0.2 * W.min_gap(W.GL, int(max(orders))) / kx / 0.3)
    wm.exact = lambda x, y, t: u0(x - c[0] * t, y - c[1] * t)
    p = _params(kx, kx, int(orders[0]))
    g, st = oracle.step_mixed(p, wm.orders, wm.initial(), a=wm.velocity(), dt=wm.dt, nsteps=nsteps)
    return wm.l2_error(g, nsteps * wm.dt), wm.l2_error(wm.initial(), 0.0)


def test_translation_accuracy_bounded_by_lowest_order():
    kx = 6
    rng = np.random.default_rng(3)
    mixed = rng.choice([6, 8, 10], size=kx * kx)
    e_mix, z = _translation_error(mixed, kx)
    e_low, _ = _translation_error(np.full(kx * kx, 6), kx)
    e_high, _ = _translation_error(np.full(kx * kx, 10), kx)
    assert z < 1e-14
    assert e_high < e_low
    assert e_mix <= 1.5 * e_low, (e_mix, e_low, e_high)
    assert e_mix < 1e-3


def test_mirror_symmetry_of_the_face_coupling():
    """Reflecting the mesh (x -> 1 - x) together with the velocity's x
    component and the element orders gives the reflected result."""
    kx, ky = 4, 4
    rng = np.random.default_rng(4)
    orders = rng.choice([5, 7, 9], size=kx * ky).reshape(ky, kx)
    u0 = lambda x, y: np.exp(-20 * ((x - 0.4) ** 2 + (y - 0.55) ** 2))
    vel = lambda x, y: (0.3 + 0.1 * np.sin(2 * math.pi * y), 0.2 + 0 * x)
    velm = lambda x, y: (-(0.3 + 0.1 * np.sin(2 * math.pi * y)), 0.2 + 0 * x)
    dt = 0.2 * W.min_gap(W.GL, 9) / kx / 0.4
    wa = _mixed(kx, ky, orders.ravel(), u0, vel, dt)
    wb = _mixed(kx, ky, orders[:, ::-1].ravel(), lambda x, y: u0(1 - x, y), velm, dt)
    p = _params(kx, ky, 5)
    ga, _ = oracle.step_mixed(p, wa.orders, wa.initial(), a=wa.velocity(), dt=dt, nsteps=2)
    gb, _ = oracle.step_mixed(p, wb.orders, wb.initial(), a=wb.velocity(), dt=dt, nsteps=2)
    # map b back: element (ix, iy) of b is element (kx-1-ix, iy) of a, node i -> n-1-i
    offa, offb = wa.offsets, wb.offsets
    for iy in range(ky):
        for ix in range(kx):
            ea, eb = iy * kx + ix, iy * kx + (kx - 1 - ix)
            n = int(wa.orders[ea])
            A = ga[offa[ea]:offa[ea + 1]].reshape(n, n)
            B = gb[offb[eb]:offb[eb + 1]].reshape(n, n)[:, ::-1]
            assert np.max(np.abs(A - B)) <= 1e-12


def test_rejects_what_it_does_not_cover():
    p = _params(2, 2, 5)
    wm = _mixed(2, 2, [5, 5, 5, 5], lambda x, y: x, W.swirl_velocity, 1e-3)
    p.cmask = W.BOUNDARY | W.MASS
    with pytest.raises(ValueError):
        oracle.step_mixed(p, wm.orders, wm.initial(), a=wm.velocity(), dt=1e-3)
    p.cmask = W.BOUNDARY
    p.bc = W.GHOST
    with pytest.raises(ValueError):
        oracle.step_mixed(p, wm.orders, wm.initial(), a=wm.velocity(), dt=1e-3)
