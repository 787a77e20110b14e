"""Seeded synthetic workloads for the semi-Lagrangian step.

This module is the one piece shared by the HIP path's tests/benchmark and by
the CPU oracle.  It holds only problem definitions -- domain, mesh, initial
field, velocity field, closed-form exact solutions and run lengths -- and
samples them at the node positions of a node family, which it takes from
numpy's library quadrature routines.  It contains none of the method's
arithmetic (no interpolation, advection, remap or constraint code).

Workloads (seed 0 unless stated):

* ``c1``  1D u_t + u_x = 0 on [0,2] periodic, K=16, order 8 (9 Gauss-Legendre
  nodes), u0 = sin(pi x), RK4, dt = 0.2 * min node gap * dx, 200 steps,
  boundary constraint only.  Exact: sin(pi (x - t)).
* ``c2``  1D a(x) = 1 + sin(pi x)/2 on [0,2] periodic, K=65536, order 16
  (17 nodes), u0 = exp(-40 (x-1)^2), RK4, boundary+mass+energy, 1000 steps.
  Exact: u0 at the foot of the characteristic (closed-form flow map).
* ``c3``  2D solid-body rotation a = (-(y-1/2), x-1/2) on [0,1]^2, 256x256
  elements, order 8 (9x9 nodes), Gaussian hill exp(-100((x-.7)^2+(y-.5)^2)),
  inflow ghost values from the exact solution, boundary constraint only.
* ``x1``, ``x6``, ``x9``: the paper's own test problems (section 5.1, 5.2, 5.3).
"""
from __future__ import annotations

import dataclasses
import math
from typing import Callable, Optional

import numpy as np

GL, CG = 0, 1
PERIODIC, GHOST = 0, 1
# 2D: periodic in x with ghost values on the bottom and top sides, or the
# other way round
PERIODIC_X, PERIODIC_Y = 2, 3
ADVECTIVE, CONSERVATIVE = 0, 1
HARD, SOFT = 0, 1
BOUNDARY, MASS, ENERGY = 1, 2, 4


def nodes(family: int, n: int) -> np.ndarray:
    """Node positions on [0,1] in ascending order (numpy library rules)."""
    if family == GL:
        t, _ = np.polynomial.legendre.leggauss(n)
    elif family == CG:
        t, _ = np.polynomial.chebyshev.chebgauss(n)
    else:
        raise ValueError(family)
    return np.sort((1.0 - t) * 0.5)


def gl_weights(n: int) -> np.ndarray:
    """Gauss-Legendre weights on [0,1], ordered like nodes(GL, n)."""
    t, w = np.polynomial.legendre.leggauss(n)
    order = np.argsort((1.0 - t) * 0.5)
    return (w * 0.5)[order]


def min_gap(family: int, n: int) -> float:
    """Smallest distance between adjacent nodes on [0,1]."""
    x = nodes(family, n)
    return float(np.min(np.diff(x))) if n > 1 else 1.0


def edge_gap(family: int, n: int) -> float:
    """Distance between the element edge and the first node (the paper's
    minimum particle spacing at the element edge, used for its time step)."""
    return float(nodes(family, n)[0])


@dataclasses.dataclass
class Workload:
    name: str
    dim: int
    kx: int
    ky: int
    n: int
    family: int
    x0: float
    x1: float
    y0: float
    y1: float
    bc: int
    form: int
    rk: int
    cmask: int
    mode: int
    dt: float
    nsteps: int
    u0: Callable
    vel: Callable                      # (x, y) -> (u, v, div)
    exact: Optional[Callable] = None   # (x, y, t) -> phi
    energy_tol: float = 1e-8
    energy_maxit: int = 50
    seed: int = 0
    vel_kind: int = 0                  # analytic id understood by the oracle

    @property
    def K(self) -> int:
        return self.kx * self.ky

    @property
    def nd(self) -> int:
        return self.n if self.dim == 1 else self.n * self.n

    @property
    def dx(self) -> float:
        return (self.x1 - self.x0) / self.kx

    @property
    def dy(self) -> float:
        return (self.y1 - self.y0) / self.ky if self.dim == 2 else 1.0

    @property
    def dofs(self) -> int:
        return self.K * self.nd

    def coords(self):
        """Physical node coordinates, element-major [K][nd]; node index i + n j
        with i along x; element index ix + kx iy."""
        xi = nodes(self.family, self.n)
        if self.dim == 1:
            ex = np.arange(self.kx)[:, None]
            x = self.x0 + (ex + xi[None, :]) * self.dx
            return x, np.zeros_like(x)
        ii, jj = np.meshgrid(np.arange(self.n), np.arange(self.n), indexing="xy")
        ii, jj = ii.ravel(), jj.ravel()  # node p = ii + n jj
        e = np.arange(self.K)
        ex, ey = e % self.kx, e // self.kx
        x = self.x0 + (ex[:, None] + xi[ii][None, :]) * self.dx
        y = self.y0 + (ey[:, None] + xi[jj][None, :]) * self.dy
        return x, y

    def initial(self) -> np.ndarray:
        x, y = self.coords()
        return np.ascontiguousarray(self.u0(x, y), dtype=np.float64).ravel()

    def velocity(self):
        """Nodal velocity, component-major [dim][K][nd], and nodal divergence."""
        x, y = self.coords()
        u, v, d = self.vel(x, y)
        u = np.broadcast_to(np.asarray(u, dtype=np.float64), x.shape)
        v = np.broadcast_to(np.asarray(v, dtype=np.float64), x.shape)
        d = np.broadcast_to(np.asarray(d, dtype=np.float64), x.shape)
        if self.dim == 1:
            a = np.ascontiguousarray(u).ravel()
        else:
            a = np.concatenate([np.ravel(u), np.ravel(v)])
        return np.ascontiguousarray(a), np.ascontiguousarray(d).ravel()

    def exact_at(self, t: float) -> np.ndarray:
        x, y = self.coords()
        return np.ascontiguousarray(self.exact(x, y, t), dtype=np.float64).ravel()

    # ghost layout: 1D [left, right]; 2D left (ky*n, by iy then node j),
    # right (ky*n), bottom (kx*n, by ix then node i), top (kx*n)
    def ghost_points(self):
        xi = nodes(self.family, self.n)
        if self.dim == 1:
            return np.array([self.x0, self.x1]), np.zeros(2)
        ys = (self.y0 + (np.arange(self.ky)[:, None] + xi[None, :]) * self.dy).ravel()
        xs = (self.x0 + (np.arange(self.kx)[:, None] + xi[None, :]) * self.dx).ravel()
        gx = np.concatenate([np.full_like(ys, self.x0), np.full_like(ys, self.x1), xs, xs])
        gy = np.concatenate([ys, ys, np.full_like(xs, self.y0), np.full_like(xs, self.y1)])
        return gx, gy

    def ghost_rows(self, t0: float, nsteps: int) -> np.ndarray:
        """Exact-solution ghost values at t0 + i dt, i = 0..nsteps (row i is
        the outside state at the start of step i, row i+1 at its end)."""
        gx, gy = self.ghost_points()
        rows = [self.exact(gx, gy, t0 + i * self.dt) for i in range(nsteps + 1)]
        return np.ascontiguousarray(np.array(rows, dtype=np.float64))

    def quad_weights(self) -> np.ndarray:
        """Physical quadrature weights per node (Gauss-Legendre only)."""
        w = gl_weights(self.n)
        if self.dim == 1:
            return np.tile(w * self.dx, self.K)
        w2 = np.outer(w, w).ravel()  # index jj*n + ii -> w[jj] w[ii]
        return np.tile(w2 * self.dx * self.dy, self.K)

    def l2_error(self, phi: np.ndarray, t: float) -> float:
        """The paper's L2 norm (eq. 5.2, physical dx): sum over elements of
        each element's L2 error, by Gauss-Legendre quadrature at the nodes."""
        err = (phi - self.exact_at(t)) ** 2 * self.quad_weights()
        return float(np.sum(np.sqrt(err.reshape(self.K, self.nd).sum(axis=1))))


# --------------------------------------------------------------------------
# analytic fields
# --------------------------------------------------------------------------
def _c2_flow_inverse_setup():
    b = 0.5
    s = math.sqrt(1.0 - b * b)
    P = 2.0 / s

    def F(x):
        """continuous antiderivative of 1/(1 + sin(pi x)/2), F(0) = G(0)"""
        m = np.floor((x + 1.0) / 2.0)
        xr = x - 2.0 * m
        G = (2.0 / (math.pi * s)) * np.arctan((np.tan(math.pi * xr / 2.0) + b) / s)
        return G + m * P

    def Finv(tau):
        m = np.round(tau / P)
        tr = tau - m * P
        xr = (2.0 / math.pi) * np.arctan(s * np.tan(math.pi * s * tr / 2.0) - b)
        return xr + 2.0 * m

    return F, Finv


_C2F, _C2Finv = _c2_flow_inverse_setup()


def c2_u0(x, y=None):
    xp = np.mod(x, 2.0)
    return np.exp(-40.0 * (xp - 1.0) ** 2)


def c2_exact(x, y, t):
    foot = _C2Finv(_C2F(np.asarray(x, dtype=np.float64)) - t)
    return c2_u0(foot)


def c3_u0(x, y):
    return np.exp(-100.0 * ((x - 0.7) ** 2 + (y - 0.5) ** 2))


def c3_exact(x, y, t):
    c, s = math.cos(t), math.sin(t)
    X, Y = x - 0.5, y - 0.5
    # foot = c + R(-t)(x - c)
    xf = 0.5 + c * X + s * Y
    yf = 0.5 - s * X + c * Y
    return c3_u0(xf, yf)


def x6_exact(x, y, t):
    """Closed-form solution of phi_t + (-sin(x) phi)_x = 0 with the paper's
    initial condition (section 5.2): c / (cos^2(x/2) + c^2 sin^2(x/2)),
    c = exp(t - 1)."""
    c = math.exp(t - 1.0)
    return c / (np.cos(x / 2.0) ** 2 + c * c * np.sin(x / 2.0) ** 2)


def c1(n: int = 9, K: int = 16, nsteps: int = 200) -> Workload:
    dx = 2.0 / K
    dt = 0.2 * min_gap(GL, n) * dx / 1.0
    return Workload(
        name="c1", dim=1, kx=K, ky=1, n=n, family=GL, x0=0.0, x1=2.0, y0=0.0, y1=1.0,
        bc=PERIODIC, form=ADVECTIVE, rk=4, cmask=BOUNDARY, mode=HARD, dt=dt, nsteps=nsteps,
        u0=lambda x, y: np.sin(math.pi * x),
        vel=lambda x, y: (np.ones_like(x), 0.0, 0.0),
        exact=lambda x, y, t: np.sin(math.pi * (x - t)),
        vel_kind=1,
    )


def c2(K: int = 65536, n: int = 17, nsteps: int = 1000, cmask: int = BOUNDARY | MASS | ENERGY) -> Workload:
    dx = 2.0 / K
    dt = 0.2 * min_gap(GL, n) * dx / 1.5
    return Workload(
        name="c2", dim=1, kx=K, ky=1, n=n, family=GL, x0=0.0, x1=2.0, y0=0.0, y1=1.0,
        bc=PERIODIC, form=ADVECTIVE, rk=4, cmask=cmask, mode=HARD, dt=dt, nsteps=nsteps,
        u0=lambda x, y: c2_u0(x),
        vel=lambda x, y: (1.0 + 0.5 * np.sin(math.pi * x), 0.0, 0.5 * math.pi * np.cos(math.pi * x)),
        exact=c2_exact,
        vel_kind=3,
    )


def c3(kx: int = 256, ky: Optional[int] = None, n: int = 9, nsteps: int = 200) -> Workload:
    ky = kx if ky is None else ky
    dx = 1.0 / kx
    dt = 0.2 * min_gap(GL, n) * min(dx, 1.0 / ky) / 0.5
    return Workload(
        name="c3", dim=2, kx=kx, ky=ky, n=n, family=GL, x0=0.0, x1=1.0, y0=0.0, y1=1.0,
        bc=GHOST, form=ADVECTIVE, rk=4, cmask=BOUNDARY, mode=HARD, dt=dt, nsteps=nsteps,
        u0=c3_u0,
        vel=lambda x, y: (-(y - 0.5), x - 0.5, 0.0),
        exact=c3_exact,
        vel_kind=4,
    )


def x1(P: int, H: int, rk: int = 1, cmask: int = BOUNDARY, mode: int = SOFT, T: float = 10.0) -> Workload:
    """Section 5.1: u = 1, sin(2 pi x) on [0,1] periodic, Chebyshev-Gauss
    nodes (n = P + 1), dt = edge gap * dx / |u|, floor(T/dt) steps."""
    n = P + 1
    dx = 1.0 / H
    dt = edge_gap(CG, n) * dx / 1.0
    return Workload(
        name="x1", dim=1, kx=H, ky=1, n=n, family=CG, x0=0.0, x1=1.0, y0=0.0, y1=1.0,
        bc=PERIODIC, form=ADVECTIVE, rk=rk, cmask=cmask, mode=mode, dt=dt,
        nsteps=int(math.floor(T / dt)),
        u0=lambda x, y: np.sin(2 * math.pi * x),
        vel=lambda x, y: (np.ones_like(x), 0.0, 0.0),
        exact=lambda x, y, t: np.sin(2 * math.pi * (x - t)),
        vel_kind=1,
    )


def x6(P: int = 6, H: int = 4, rk: int = 1, cmask: int = BOUNDARY, mode: int = SOFT, T: float = 1.0) -> Workload:
    """Section 5.2: phi_t + (-sin(x) phi)_x = 0 on [0, 2 pi] periodic."""
    n = P + 1
    dx = 2 * math.pi / H
    dt = edge_gap(CG, n) * dx / 1.0
    return Workload(
        name="x6", dim=1, kx=H, ky=1, n=n, family=CG, x0=0.0, x1=2 * math.pi, y0=0.0, y1=1.0,
        bc=PERIODIC, form=CONSERVATIVE, rk=rk, cmask=cmask, mode=mode, dt=dt,
        nsteps=int(math.floor(T / dt)),
        u0=lambda x, y: x6_exact(x, y, 0.0),
        vel=lambda x, y: (-np.sin(x), 0.0, -np.cos(x)),
        exact=x6_exact,
        vel_kind=2,
    )


def x9(P: int, H: int, rk: int = 1, cmask: int = BOUNDARY, mode: int = SOFT, T: float = 1.0,
       family: int = CG) -> Workload:
    """Section 5.3: a = 2, b = 1, sin(2 pi x) sin(2 pi y) on [0,1]^2 periodic."""
    n = P + 1
    dx = 1.0 / H
    dt = edge_gap(family, n) * dx / 2.0
    return Workload(
        name="x9", dim=2, kx=H, ky=H, n=n, family=family, x0=0.0, x1=1.0, y0=0.0, y1=1.0,
        bc=PERIODIC, form=ADVECTIVE, rk=rk, cmask=cmask, mode=mode, dt=dt,
        nsteps=int(math.floor(T / dt)),
        u0=lambda x, y: np.sin(2 * math.pi * x) * np.sin(2 * math.pi * y),
        vel=lambda x, y: (2.0 * np.ones_like(x), np.ones_like(x), 0.0),
        exact=lambda x, y, t: np.sin(2 * math.pi * (x - 2 * t)) * np.sin(2 * math.pi * (y - t)),
        vel_kind=1,
    )


def random_field_1d(K: int, n: int, seed: int, family: int = GL, x0: float = 0.0, x1: float = 1.0):
    """Seeded smooth random nodal field: a few Fourier modes sampled at nodes."""
    rng = np.random.default_rng(seed)
    xi = nodes(family, n)
    dx = (x1 - x0) / K
    x = x0 + (np.arange(K)[:, None] + xi[None, :]) * dx
    L = x1 - x0
    f = np.zeros_like(x)
    for _ in range(4):
        k = rng.integers(1, 4)
        f += rng.normal() * np.sin(2 * math.pi * k * (x - x0) / L + rng.uniform(0, 2 * math.pi))
    return np.ascontiguousarray(f.ravel())


def random_field_2d(kx: int, ky: int, n: int, seed: int, modes: int = 8, family: int = GL):
    """u0 = sum of `modes` unit-amplitude sin(2 pi (p x + q y) + theta) on [0,1]^2."""
    rng = np.random.default_rng(seed)
    xi = nodes(family, n)
    ii, jj = np.meshgrid(np.arange(n), np.arange(n), indexing="xy")
    ii, jj = ii.ravel(), jj.ravel()
    e = np.arange(kx * ky)
    x = (e[:, None] % kx + xi[ii][None, :]) / kx
    y = (e[:, None] // kx + xi[jj][None, :]) / ky
    f = np.zeros_like(x)
    for _ in range(modes):
        while True:
            p, q = rng.integers(-4, 5, size=2)
            if p or q:
                break
        f += np.sin(2 * math.pi * (p * x + q * y) + rng.uniform(0, 2 * math.pi))
    return np.ascontiguousarray(f.ravel())


# ---------------------------------------------------------------------------
# Mixed orders in 2D: every element has its own number of nodes n_e per
# direction.  Arrays are concatenated element by element (e = ix + kx*iy),
# n_e^2 values each, node i + n_e j with i along x; a velocity array holds
# all u values, then all v values.
# ---------------------------------------------------------------------------
@dataclasses.dataclass
class MixedWorkload:
    name: str
    kx: int
    ky: int
    orders: np.ndarray              # [K] nodes per direction per element
    family: int
    dt: float
    nsteps: int
    u0: Callable                    # (x, y) -> phi
    vel: Callable                   # (x, y) -> (u, v)
    mode: int = HARD
    form: int = ADVECTIVE
    rk: int = 4
    x0: float = 0.0
    x1: float = 1.0
    y0: float = 0.0
    y1: float = 1.0
    exact: Optional[Callable] = None  # (x, y, t) -> phi

    @property
    def K(self) -> int:
        return self.kx * self.ky

    @property
    def dofs(self) -> int:
        return int((self.orders.astype(np.int64) ** 2).sum())

    @property
    def offsets(self) -> np.ndarray:
        return np.concatenate([[0], np.cumsum(self.orders.astype(np.int64) ** 2)])

    def coords(self):
        dx = (self.x1 - self.x0) / self.kx
        dy = (self.y1 - self.y0) / self.ky
        xs, ys = [], []
        cache = {}
        for e, n in enumerate(self.orders):
            n = int(n)
            if n not in cache:
                xi = nodes(self.family, n)
                ii, jj = np.meshgrid(np.arange(n), np.arange(n), indexing="xy")
                cache[n] = (xi[ii.ravel()], xi[jj.ravel()])
            sx, sy = cache[n]
            xs.append(self.x0 + (e % self.kx + sx) * dx)
            ys.append(self.y0 + (e // self.kx + sy) * dy)
        return np.concatenate(xs), np.concatenate(ys)

    def initial(self):
        x, y = self.coords()
        return np.ascontiguousarray(self.u0(x, y), dtype=np.float64)

    def velocity(self):
        x, y = self.coords()
        u, v = self.vel(x, y)
        return np.ascontiguousarray(np.concatenate([np.broadcast_to(u, x.shape), np.broadcast_to(v, x.shape)]))

    def exact_at(self, t):
        x, y = self.coords()
        return self.exact(x, y, t)

    def l2_error(self, phi, t):
        """Sum over elements of each element's physical L2 error (the paper's
        norm, eq. 5.2), element by element with its own quadrature."""
        x, y = self.coords()
        err = np.asarray(phi) - self.exact(x, y, t)
        dx = (self.x1 - self.x0) / self.kx
        dy = (self.y1 - self.y0) / self.ky
        off = self.offsets
        tot = 0.0
        wcache = {}
        for e, n in enumerate(self.orders):
            n = int(n)
            if n not in wcache:
                wq = gl_weights(n) if self.family == GL else np.full(n, 1.0 / n)
                wcache[n] = np.outer(wq, wq).ravel()
            d = err[off[e]:off[e + 1]]
            tot += math.sqrt(dx * dy * float(np.dot(wcache[n], d * d)))
        return tot


def swirl_velocity(x, y):
    """a = (sin^2(pi x) sin(2 pi y), -sin^2(pi y) sin(2 pi x)): divergence
    free, zero normal component on the walls of [0,1]^2, periodic."""
    sx, sy = np.sin(math.pi * x), np.sin(math.pi * y)
    return sx * sx * np.sin(2 * math.pi * y), -sy * sy * np.sin(2 * math.pi * x)


def fourier_modes(seed: int, modes: int = 8):
    """u0 = sum of `modes` unit-amplitude sin(2 pi (p x + q y) + theta), with
    integers (p, q) in [-4, 4]^2 minus the origin and theta uniform, by seed."""
    rng = np.random.default_rng(seed)
    terms = []
    for _ in range(modes):
        while True:
            p, q = rng.integers(-4, 5, size=2)
            if p or q:
                break
        terms.append((int(p), int(q), float(rng.uniform(0, 2 * math.pi))))
    return lambda x, y: sum(np.sin(2 * math.pi * (p * x + q * y) + th) for p, q, th in terms)


def c4(kx: int = 316, ky: Optional[int] = None, nsteps: int = 100, seed: int = 0,
       orders=(4, 6, 8, 12)) -> MixedWorkload:
    """Mixed-order batch: kx x ky quads on [0,1]^2 (316 x 316 = 99,856 by
    default), per-element order drawn from `orders` by seed, swirl velocity,
    eight random Fourier modes, periodic, boundary rows (HARD), RK4,
    dt = 0.2 * (min node spacing of the largest order) * dx / max |a|."""
    ky = kx if ky is None else ky
    rng = np.random.default_rng(seed)
    n_e = np.asarray(orders)[rng.integers(0, len(orders), size=kx * ky)] + 1
    nmax = int(max(orders)) + 1
    dt = 0.2 * min_gap(GL, nmax) * (1.0 / max(kx, ky)) / 1.0
    return MixedWorkload(name="c4", kx=kx, ky=ky, orders=n_e.astype(np.int32), family=GL, dt=dt, nsteps=nsteps,
                         u0=fourier_modes(seed + 1), vel=swirl_velocity)
