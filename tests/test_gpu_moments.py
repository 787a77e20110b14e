"""The global mass and energy that sl_read reports (sl_stats.mass, .energy):
the quadrature sums of phi and phi^2 with the node weights times the element
size (section 4, mass and energy conservation), reduced on the device.  They
must equal the same sums taken here in numpy over the field the same read
returns, for 1D, 2D and mixed-order meshes; and a read between steps must
leave the later steps unchanged, bit for bit."""
import numpy as np
import pytest

import oracle
import workloads as W
from _parity import announce, opts_dict

pytestmark = pytest.mark.gpu
TOL = 1e-13


@pytest.fixture(scope="module", autouse=True)
def _need_gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1910_06476_amd as P
    P.lib()


def _weights(family, n, dim):
    _, wq = oracle.nodes(family, n)
    return wq if dim == 1 else np.outer(wq, wq).ravel()


def _sums(field, ns, family, dim, h):
    """Mass, energy and the scale sum |w phi| of a field whose element e has
    ns[e] nodes per direction, element-major."""
    M = E = S = 0.0
    off = 0
    cache = {}
    for n in ns:
        nd = n if dim == 1 else n * n
        if n not in cache:
            cache[n] = _weights(family, n, dim)
        v = field[off:off + nd]
        w = cache[n]
        M += (w * v).sum()
        E += (w * v * v).sum()
        S += (w * np.abs(v)).sum()
        off += nd
    assert off == field.size
    return M * h, E * h, S * h


def _check(st, field, ns, family, dim, h):
    M, E, S = _sums(np.asarray(field), ns, family, dim, h)
    assert abs(st.mass - M) <= TOL * S, (st.mass, M)
    assert abs(st.energy - E) <= TOL * E, (st.energy, E)


def _uniform(w, split):
    """Steps run in one call, or split in two with a read in between: the
    final fields must be the same bit for bit; returns both reads."""
    import paper_1910_06476_amd as P
    m = P.from_workload(w)
    try:
        if w.bc == W.GHOST:
            m.set_ghost(w.ghost_rows(0.0, w.nsteps))
        opts = opts_dict(w)
        reads = []
        if split:
            m.step(w.dt, 2, **opts)
            reads.append(m.read())
            m.step(w.dt, w.nsteps - 2, **opts)
        else:
            m.step(w.dt, w.nsteps, **opts)
        reads.append(m.read())
    finally:
        m.close()
    return reads


@pytest.mark.parametrize("case", ["1d", "2d"])
def test_mass_and_energy_of_uniform_meshes(case):
    w = W.c2(K=300, n=9, nsteps=5) if case == "1d" else W.c3(kx=11, n=7, nsteps=5)
    announce(f"moments {case} K={w.K} n={w.n}")
    h = w.dx if w.dim == 1 else w.dx * w.dy
    ns = [w.n] * w.K
    whole = _uniform(w, False)
    split = _uniform(w, True)
    for rc, field, st in split + whole:
        assert rc == 0
        _check(st, field, ns, w.family, w.dim, h)
    assert np.array_equal(np.asarray(split[-1][1]), np.asarray(whole[-1][1]))


def test_mass_and_energy_of_a_mixed_mesh():
    import paper_1910_06476_amd as P
    w = W.c4(kx=12, nsteps=3)
    announce(f"moments mixed 12x12 {sorted(set(w.orders.tolist()))}")
    m = P.from_mixed_workload(w)
    try:
        m.step(w.dt, w.nsteps, rk=w.rk, constraints=W.BOUNDARY, mode=w.mode)
        rc, field, st = m.read()
    finally:
        m.close()
    assert rc == 0
    h = (w.x1 - w.x0) / w.kx * (w.y1 - w.y0) / w.ky
    _check(st, field, [int(n) for n in w.orders], w.family, 2, h)
