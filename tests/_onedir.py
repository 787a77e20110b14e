"""Inputs of the one-direction-periodic cases (2D), shared by the oracle pin
and the GPU check: a polynomial in the coordinate across the ghost sides,
constant along the periodic direction, moved by a constant velocity, so the
exact solution is the shifted polynomial.  The ghost rows hold the exact
solution on the ghost sides and NaN on the periodic sides, which must never
be read."""
import numpy as np

import workloads as W


def case(bc: int, deg: int, cmask: int = W.BOUNDARY, mode: int = W.HARD, n: int = 5, nsteps: int = 3,
         form: int = W.ADVECTIVE):
    a, b = 0.7, -0.4
    rng = np.random.default_rng(deg + 7 * n + 31 * bc)
    c = rng.normal(size=deg + 1)
    if bc == W.PERIODIC_X:  # varies across the bottom and top (ghost) sides
        f = lambda x, y, t: np.polynomial.polynomial.polyval(y - b * t, c) + 0.0 * x
    else:
        f = lambda x, y, t: np.polynomial.polynomial.polyval(x - a * t, c) + 0.0 * y
    kx, ky = 3, 2
    w = W.Workload(name="onedir", dim=2, kx=kx, ky=ky, n=n, family=W.GL, x0=-0.3, x1=1.2, y0=0.1, y1=0.9,
                   bc=bc, form=form, rk=4, cmask=cmask, mode=mode, dt=0.2 * W.min_gap(W.GL, n) * 0.4 / 0.7,
                   nsteps=nsteps, u0=lambda x, y: f(x, y, 0.0),
                   vel=lambda x, y: (a * np.ones_like(x), b * np.ones_like(x), 0.0), exact=f,
                   energy_tol=0.0, energy_maxit=6)
    g = w.ghost_rows(0.0, nsteps)
    KL, KB = ky * n, kx * n
    if bc == W.PERIODIC_X:
        g[:, :2 * KL] = np.nan  # left and right sides wrap
    else:
        g[:, 2 * KL:2 * KL + 2 * KB] = np.nan  # bottom and top sides wrap
    return w, g
