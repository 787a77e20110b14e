"""Inputs and closed-form result of the linear-velocity step, shared by the
oracle pin and the GPU check (no arithmetic of the method here).

For a = c x (2D: a = (c x, c y)) every Runge-Kutta stage is affine in the
position, so one step of an explicit s-stage method moves each particle to
R(c dt) x exactly, R the method's stability function; for the tableaux of
order s <= 4 used here, R is the degree-s Taylor polynomial of e^z.  The
field u0 = x (2D: x + y) is carried to those points and remapped exactly
(degree 1), giving u = u0 / R(c dt).  In the conservative form the carried
values obey dq/dt = -q div a = -d c q (d the dimension), so they become
R(-d c dt) q and u = R(-d c dt) / R(c dt) u0.  No constraint rows are
imposed, so the step returns the remap itself."""
import math

import numpy as np

import workloads as W


def stability(z: float, s: int) -> float:
    return sum(z ** k / math.factorial(k) for k in range(s + 1))


def case(dim: int, rk: int, form: int, n: int = 3, c: float = 0.9):
    """Workload (GHOST boundaries, zero ghost rows, no constraint rows), the
    nodal velocity [dim][K][nd] and divergence, and the expected field."""
    kx, ky = (3, 1) if dim == 1 else (2, 2)
    x0 = y0 = 0.1
    dx = 0.5
    x1, y1 = x0 + kx * dx, (y0 + ky * dx if dim == 2 else 1.0)
    xi = W.nodes(W.GL, n)
    dt = 0.8 * xi[0] * dx / (c * max(x1, y1))  # every particle stays in its element
    vel = (lambda x, y: (c * x, 0.0, c)) if dim == 1 else (lambda x, y: (c * x, c * y, 2.0 * c))
    u0 = (lambda x, y: x) if dim == 1 else (lambda x, y: x + y)
    w = W.Workload(name="linear", dim=dim, kx=kx, ky=ky, n=n, family=W.GL, x0=x0, x1=x1, y0=y0,
                   y1=y1 if dim == 2 else 1.0, bc=W.GHOST, form=form, rk=rk, cmask=0, mode=W.HARD, dt=dt,
                   nsteps=1, u0=u0, vel=vel, exact=None)
    a, div = w.velocity()
    z = c * dt
    f0 = w.initial()
    if form == W.ADVECTIVE:
        expect = f0 / stability(z, rk)
    else:
        expect = stability(-dim * z, rk) / stability(z, rk) * f0
    gx, _ = w.ghost_points()
    ghost = np.zeros((2, gx.size))
    return w, a, div, ghost, expect
