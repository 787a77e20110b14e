"""Inputs of the zero-velocity cases, shared by the oracle pin and the GPU
check: with a = 0 no particle moves and every face speed is zero, so every
face takes the tie rule (the mean of the two traces).  A field that is one
polynomial of degree <= N over the whole domain, with its own values as the
ghost rows, has equal traces on both sides of every face and must come back
unchanged; a periodic field that is not a polynomial exercises the tie rule
between unequal traces."""
import math

import numpy as np

import workloads as W


def polynomial_case(dim: int, cmask: int, mode: int = W.HARD):
    if dim == 1:
        f = lambda x, y, t: 0.3 + 0.5 * x - 0.2 * x ** 3
    else:
        f = lambda x, y, t: 0.3 + 0.5 * x * y - 0.2 * y ** 3 + x ** 2
    return W.Workload(name="zerovel", dim=dim, kx=5 if dim == 1 else 3, ky=1 if dim == 1 else 2, n=5,
                      family=W.GL, x0=-0.3, x1=1.2, y0=0.1, y1=0.9 if dim == 2 else 1.0, bc=W.GHOST,
                      form=W.ADVECTIVE, rk=4, cmask=cmask, mode=mode, dt=1e-3, nsteps=3,
                      u0=lambda x, y: f(x, y, 0.0), vel=lambda x, y: (0.0 * x, 0.0 * x, 0.0), exact=f,
                      energy_tol=0.0, energy_maxit=3)


def periodic_case(dim: int, cmask: int, mode: int = W.HARD):
    f = (lambda x, y, t: np.exp(np.sin(2 * math.pi * x))) if dim == 1 else \
        (lambda x, y, t: np.exp(np.sin(2 * math.pi * x) * np.cos(2 * math.pi * y)))
    return W.Workload(name="zerovel_p", dim=dim, kx=6 if dim == 1 else 4, ky=1 if dim == 1 else 3, n=6,
                      family=W.GL, x0=0.0, x1=1.0, y0=0.0, y1=1.0, bc=W.PERIODIC, form=W.ADVECTIVE, rk=4,
                      cmask=cmask, mode=mode, dt=1e-3, nsteps=3, u0=lambda x, y: f(x, y, 0.0),
                      vel=lambda x, y: (0.0 * x, 0.0 * x, 0.0), exact=f, energy_tol=0.0, energy_maxit=3)
