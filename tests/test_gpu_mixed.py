"""GPU parity of mixed-order 2D meshes (per-element orders, periodic,
boundary rows) against the oracle's mixed-order step, through the C-ABI.
The device runs the order buckets as separate launches, captured in a HIP
graph, with block shapes picked by the autotuner; none of that may change a
result.  Bar: relative L2 <= 1e-12 (FP64)."""
import math

import numpy as np
import pytest

import oracle
import workloads as W
from _parity import announce, rel_l2

pytestmark = pytest.mark.gpu
TOL = 1e-12


@pytest.fixture(scope="module", autouse=True)
def _need_gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1910_06476_amd as P
    P.lib()


def _case(kx, ky, orders, seed=0, mode=W.HARD, form=W.ADVECTIVE, nsteps=3):
    w = W.c4(kx=kx, ky=ky, nsteps=nsteps, seed=seed, orders=orders)
    w.mode, w.form = mode, form
    return w


def _gpu(w, nsteps=None, profiling=False, precision=0):
    import paper_1910_06476_amd as P
    m = P.from_mixed_workload(w, precision=precision)
    try:
        if profiling:
            P.sl_set_profiling(m.h, True)
        m.step(w.dt, w.nsteps if nsteps is None else nsteps, rk=w.rk, constraints=W.BOUNDARY, mode=w.mode)
        rc, out, st = m.read()
    finally:
        m.close()
    return out, st, rc


def _oracle(w, nsteps=None):
    p = oracle.Params(dim=2, kx=w.kx, ky=w.ky, n=int(w.orders[0]), family=w.family, bc=W.PERIODIC, form=w.form,
                      rk=w.rk, cmask=W.BOUNDARY, mode=w.mode, energy_maxit=0, vel_kind=0, x0=w.x0, x1=w.x1,
                      y0=w.y0, y1=w.y1, energy_tol=0.0)
    return oracle.step_mixed(p, w.orders, w.initial(), a=w.velocity(), dt=w.dt,
                             nsteps=w.nsteps if nsteps is None else nsteps)


@pytest.mark.parametrize("mode", [W.HARD, W.SOFT])
@pytest.mark.parametrize("form", [W.ADVECTIVE, W.CONSERVATIVE])
def test_c4_orders_parity(mode, form):
    w = _case(6, 5, (4, 6, 8, 12), seed=1, mode=mode, form=form)
    announce(f"mixed c4 orders mode={mode} form={form}")
    g, st, rc = _gpu(w)
    o, ost = _oracle(w)
    assert rc == 0 and (st.flags & ~2) == 0, (rc, st.flags)
    assert rel_l2(g, o) <= TOL, rel_l2(g, o)


@pytest.mark.parametrize("precision", [1, 2])
def test_c4_orders_reduced_precision_preconditioner_parity(precision):
    """FP32 and BF16 remap preconditioners on a mixed-order mesh: FP64
    residuals, so the same FP64 solution."""
    w = _case(6, 5, (4, 6, 8, 12), seed=4)
    announce(f"mixed c4 orders precision={precision}")
    g, st, rc = _gpu(w, precision=precision)
    o, ost = _oracle(w)
    assert rc == 0 and (st.flags & ~2) == 0, (rc, st.flags)
    assert rel_l2(g, o) <= TOL, rel_l2(g, o)


@pytest.mark.parametrize("seed", [2, 3])
def test_all_orders_parity(seed):
    """Orders drawn from 1..16 on 64 elements: up to sixteen buckets (order
    16 with 289 particles per element in 320-lane blocks) and the
    interpolation matrices between every pair present."""
    w = _case(8, 8, tuple(range(1, 17)), seed=seed, nsteps=2)
    announce(f"mixed all orders seed={seed}")
    g, st, rc = _gpu(w)
    o, ost = _oracle(w)
    assert rc == 0
    assert rel_l2(g, o) <= TOL, rel_l2(g, o)


@pytest.mark.parametrize("nsteps", [1, 2, 5])
def test_graph_replay_equals_eager(nsteps):
    """Profiling forces the eager path; the graph path must give the same
    bits, also over several replays and an odd final step."""
    w = _case(5, 5, (4, 6, 8, 12), seed=4, nsteps=nsteps)
    announce(f"mixed graph vs eager nsteps={nsteps}")
    g1, _, _ = _gpu(w, profiling=True)
    g2, _, _ = _gpu(w)
    assert np.array_equal(g1, g2)


@pytest.mark.parametrize("order", [8, 12])
def test_uniform_orders_match_the_uniform_mesh(order):
    """All elements of one order through the mixed path equal the uniform
    mesh bit for bit (same arithmetic, other launches; an element's result
    does not depend on the block shape, order 12 takes another shape on the
    uniform mesh than order 8)."""
    import paper_1910_06476_amd as P
    w = _case(5, 4, (order,), seed=5)
    announce("mixed uniform vs uniform mesh")
    g, _, _ = _gpu(w)
    n = int(w.orders[0])
    m = P.Mesh(2, w.kx, w.ky, n - 1, w.initial(), nodes=w.family, bc=P.SL_BC_PERIODIC, form=w.form)
    try:
        m.set_velocity(w.velocity())
        m.step(w.dt, w.nsteps, rk=w.rk, constraints=W.BOUNDARY, mode=w.mode)
        rc, u, st = m.read()
    finally:
        m.close()
    assert np.array_equal(g, u)


def test_velocity_change_right_after_steps():
    """A new velocity set right after sl_step, with no read in between, must
    not change the steps already queued: two graph replays (four steps) with
    the velocity a, then four steps with a / 2, equal the oracle run in the
    same two legs."""
    import paper_1910_06476_amd as P
    w = _case(6, 5, (4, 6, 8, 12), seed=6, nsteps=4)
    announce("mixed velocity change after steps")
    a1 = w.velocity()
    a2 = 0.5 * a1
    m = P.from_mixed_workload(w)
    try:
        m.step(w.dt, 4, rk=w.rk, constraints=W.BOUNDARY, mode=w.mode)
        m.set_velocity(a2)
        m.step(w.dt, 4, rk=w.rk, constraints=W.BOUNDARY, mode=w.mode)
        rc, g, st = m.read()
    finally:
        m.close()
    p = oracle.Params(dim=2, kx=w.kx, ky=w.ky, n=int(w.orders[0]), family=w.family, bc=W.PERIODIC, form=w.form,
                      rk=w.rk, cmask=W.BOUNDARY, mode=w.mode, energy_maxit=0, vel_kind=0, x0=w.x0, x1=w.x1,
                      y0=w.y0, y1=w.y1, energy_tol=0.0)
    o, _ = oracle.step_mixed(p, w.orders, w.initial(), a=a1, dt=w.dt, nsteps=4)
    o, _ = oracle.step_mixed(p, w.orders, o, a=a2, dt=w.dt, nsteps=4)
    assert rc == 0
    assert rel_l2(g, o) <= TOL, rel_l2(g, o)


def test_c4_submesh_accuracy_and_parity():
    """A 32x32 piece of the C4 recipe (orders {4,6,8,12}, swirl, eight
    Fourier modes), five steps: oracle parity of the whole field."""
    w = _case(32, 32, (4, 6, 8, 12), seed=0, nsteps=5)
    announce("mixed c4 32x32")
    g, st, rc = _gpu(w)
    o, ost = _oracle(w)
    assert rc == 0
    assert rel_l2(g, o) <= TOL, rel_l2(g, o)


def test_c4_full_size_sampled_parity():
    """Full size (316x316, orders {4,6,8,12} by seed, 8.08 M DOF) in the
    launch configuration the benchmark times: order buckets in one captured
    graph, block shapes from the autotuner.  Two steps (one graph replay).
    With boundary rows only, an element's value after two steps depends on
    the elements within two of it, so 48 seeded elements are each compared
    with the oracle run on the 5x5 window of elements around it (periodic
    within the window; the centre's dependencies are all inside)."""
    w = _case(316, 316, (4, 6, 8, 12), seed=0, nsteps=2)
    announce("mixed c4 full size, sampled")
    g, st, rc = _gpu(w)
    assert rc == 0
    off = w.offsets
    phi0 = w.initial()
    a = w.velocity()
    u, v = a[:w.dofs], a[w.dofs:]
    dx, dy = (w.x1 - w.x0) / w.kx, (w.y1 - w.y0) / w.ky
    rng = np.random.default_rng(11)
    G, O = [], []
    for e in rng.choice(w.K, 48, replace=False):
        ex, ey = int(e) % w.kx, int(e) // w.kx
        idx = [((ey + j) % w.ky) * w.kx + (ex + i) % w.kx for j in range(-2, 3) for i in range(-2, 3)]
        orders = w.orders[idx]
        cut = lambda arr: np.concatenate([arr[off[k]:off[k + 1]] for k in idx])
        p = oracle.Params(dim=2, kx=5, ky=5, n=int(orders[0]), family=w.family, bc=W.PERIODIC, form=w.form,
                          rk=w.rk, cmask=W.BOUNDARY, mode=w.mode, energy_maxit=0, vel_kind=0, x0=0.0,
                          x1=5 * dx, y0=0.0, y1=5 * dy, energy_tol=0.0)
        o, _ = oracle.step_mixed(p, orders, cut(phi0), a=np.concatenate([cut(u), cut(v)]), dt=w.dt, nsteps=2)
        sub = np.concatenate([[0], np.cumsum(orders.astype(np.int64) ** 2)])
        G.append(g[off[e]:off[e + 1]])
        O.append(o[sub[12]:sub[13]])
    err = rel_l2(np.concatenate(G), np.concatenate(O))
    assert err <= TOL, err


def test_mixed_statistics_and_validation():
    import paper_1910_06476_amd as P
    w = _case(4, 4, (4, 6), seed=6, nsteps=2)
    announce("mixed validation")
    m = P.from_mixed_workload(w)
    try:
        with pytest.raises(P.SLError) as e:  # mass rows are not offered on mixed meshes
            m.step(w.dt, 1, constraints=W.BOUNDARY | W.MASS)
        assert e.value.status == P.SL_E_INVALID
        m.step(w.dt, 2)
        rc, out, st = m.read()
        assert rc == 0 and st.steps == 2 and out.size == w.dofs
        assert st.remap_sweeps_max >= 1
    finally:
        m.close()
    with pytest.raises(P.SLError):  # ghost boundaries are not offered on mixed meshes
        P.Mesh(2, 2, 2, 3, np.zeros(4 * 16), bc=P.SL_BC_GHOST, orders=[3, 3, 3, 3])
    with pytest.raises(P.SLError):  # order 17 is beyond the 2D limit
        P.Mesh(2, 2, 2, 3, np.zeros(3 * 16 + 18 * 18), orders=[3, 3, 3, 17])
    with pytest.raises(P.SLError):  # order 16 runs in FP64 only
        P.Mesh(2, 2, 2, 3, np.zeros(3 * 16 + 17 * 17), orders=[3, 3, 3, 16], precision=P.SL_PREC_FP32_REFINED)


def test_distinct_meshes_step_concurrently():
    """Distinct meshes may be stepped from several host threads at once (the
    C-ABI's thread-safety rule): a mixed-order mesh (graph capture per
    thread), a uniform 2D mesh and a 1D mesh, each stepped in its own thread,
    give bit for bit the results of the same meshes stepped one after
    another."""
    import threading
    import paper_1910_06476_amd as P
    from _parity import run_gpu
    wm = _case(8, 6, (4, 6, 8, 12), seed=4, nsteps=6)
    w2 = W.c3(kx=12, n=7, nsteps=6)
    w1 = W.c2(K=300, nsteps=6)
    announce("concurrent meshes")

    def mixed():
        g, st, rc = _gpu(wm)
        return g

    def uni2():
        return run_gpu(w2)[0]

    def uni1():
        return run_gpu(w1)[0]

    jobs = [mixed, uni2, uni1]
    ref = [f() for f in jobs]
    out = [None] * len(jobs)
    errs = []

    def runner(i):
        try:
            for _ in range(3):
                r = jobs[i]()
                if out[i] is None:
                    out[i] = r
                elif not np.array_equal(out[i], r):
                    errs.append(i)
        except Exception as e:  # reported below
            errs.append(repr(e))

    th = [threading.Thread(target=runner, args=(i,)) for i in range(len(jobs))]
    for t in th:
        t.start()
    for t in th:
        t.join()
    assert not errs, errs
    for r, o in zip(ref, out):
        assert np.array_equal(r, o)
