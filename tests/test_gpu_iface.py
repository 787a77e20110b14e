"""GPU parity of the backtracking interface values (SL_IFACE_BACKTRACK,
eq. 4.11) against the oracle, through the C-ABI, 1D and 2D.

The velocity fields change sign inside the domain, so every case has faces
where the flow leaves through the left and through the right edge, and the
backtraces start from both edges.  Bar: relative L2 <= 1e-12 (FP64);
mass+energy HARD cases are held to the same whole-field bar."""
import math

import numpy as np
import pytest

import workloads as W
from _parity import announce, assert_parity, rel_l2, run_gpu, run_oracle

pytestmark = pytest.mark.gpu
TOL = 1e-12
BT = 1  # SL_IFACE_BACKTRACK


@pytest.fixture(scope="module", autouse=True)
def _need_gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1910_06476_amd as P
    P.lib()


def _case1d(n=7, K=37, rk=4, cmask=W.BOUNDARY, mode=W.HARD, form=W.ADVECTIVE, bc=W.PERIODIC, seed=0):
    rng = np.random.default_rng(seed)
    ph = rng.uniform(0.2, 0.5)
    f0 = lambda x: 1.2 + np.sin(2 * np.pi * x) + 0.3 * np.cos(6 * np.pi * x + ph)
    amax = 0.95
    dt = 0.2 * W.min_gap(W.GL, n) / K / amax
    return W.Workload(name="bt1", dim=1, kx=K, ky=1, n=n, family=W.GL, x0=0.0, x1=1.0, y0=0, y1=1, bc=bc,
                      form=form, rk=rk, cmask=cmask, mode=mode, dt=dt, nsteps=3,
                      u0=lambda x, y: f0(x),
                      vel=lambda x, y: (0.3 + 0.6 * np.sin(2 * np.pi * x + ph), 0.0, 0.0),
                      exact=lambda x, y, t: f0(x - 0.3 * t),  # inflow data for the ghost rows
                      energy_tol=0.0, energy_maxit=3)


def _case2d(kx, ky, n, bc=W.PERIODIC, form=W.ADVECTIVE, mode=W.HARD, rk=4, cmask=W.BOUNDARY, seed=0):
    rng = np.random.default_rng(seed)
    ph = rng.uniform(0, 2 * math.pi, 4)
    u = lambda x, y: 0.2 + 0.5 * np.sin(2 * math.pi * y + ph[0]) + 0.2 * np.cos(2 * math.pi * x + ph[1])
    v = lambda x, y: -0.1 + 0.5 * np.cos(2 * math.pi * x + ph[2]) + 0.2 * np.sin(2 * math.pi * y + ph[3])
    f0 = lambda x, y: 1.3 + np.sin(2 * math.pi * x) * np.cos(2 * math.pi * y + 0.3) + 0.2 * np.cos(4 * math.pi * x)
    dt = 0.2 * W.min_gap(W.GL, n) * min(1.0 / kx, 1.0 / ky) / 1.0
    return W.Workload(name="bt2", dim=2, kx=kx, ky=ky, n=n, family=W.GL, x0=0.0, x1=1.0, y0=0.0, y1=1.0,
                      bc=bc, form=form, rk=rk, cmask=cmask, mode=mode, dt=dt, nsteps=3,
                      energy_maxit=3, energy_tol=0.0, u0=f0, vel=lambda x, y: (u(x, y), v(x, y), 0.0),
                      exact=lambda x, y, t: f0(x - 0.2 * t, y + 0.1 * t))  # inflow data for the ghost rows


@pytest.mark.parametrize("bc", [W.PERIODIC, W.GHOST])
@pytest.mark.parametrize("form", [W.ADVECTIVE, W.CONSERVATIVE])
@pytest.mark.parametrize("cmask", [W.BOUNDARY, W.BOUNDARY | W.MASS | W.ENERGY])
@pytest.mark.parametrize("rk", [2, 4])
def test_backtrack_1d_parity(rk, cmask, form, bc):
    w = _case1d(rk=rk, cmask=cmask, form=form, bc=bc)
    announce(f"1d backtrack rk={rk} cmask={cmask} form={form} bc={bc}")
    g, st, rc = run_gpu(w, iface=BT)
    o, ost = run_oracle(w, iface=BT)
    assert_parity(w, g, o)
    assert (st.flags & ~8) == (ost.flags & ~8), (st.flags, ost.flags)


@pytest.mark.parametrize("n", [2, 5, 9, 17])
@pytest.mark.parametrize("K", [1, 16, 47])
def test_backtrack_1d_orders_and_sizes(n, K):
    cmask = W.BOUNDARY | W.MASS if n >= 3 else W.BOUNDARY
    w = _case1d(n=n, K=K, cmask=cmask, bc=W.GHOST)
    announce(f"1d backtrack n={n} K={K}")
    g, st, rc = run_gpu(w, iface=BT)
    o, ost = run_oracle(w, iface=BT)
    assert_parity(w, g, o)


@pytest.mark.parametrize("bc", [W.PERIODIC, W.GHOST, W.PERIODIC_X, W.PERIODIC_Y])
@pytest.mark.parametrize("form", [W.ADVECTIVE, W.CONSERVATIVE])
@pytest.mark.parametrize("cmask", [W.BOUNDARY, W.BOUNDARY | W.MASS])
@pytest.mark.parametrize("n", [3, 5, 9])
def test_backtrack_2d_parity(n, cmask, form, bc):
    w = _case2d(4, 3, n, bc=bc, form=form, cmask=cmask)
    announce(f"2d backtrack n={n} cmask={cmask} form={form} bc={bc}")
    g, st, rc = run_gpu(w, iface=BT)
    o, ost = run_oracle(w, iface=BT)
    assert rel_l2(g, o) <= TOL, rel_l2(g, o)
    assert (st.flags & ~8) == (ost.flags & ~8), (st.flags, ost.flags)


def test_backtrack_2d_soft_energy_parity():
    w = _case2d(3, 4, 7, mode=W.SOFT, cmask=W.BOUNDARY | W.MASS | W.ENERGY)
    announce("2d backtrack soft B+M+E")
    g, st, rc = run_gpu(w, iface=BT)
    o, ost = run_oracle(w, iface=BT)
    assert rel_l2(g, o) <= TOL, rel_l2(g, o)


def test_backtrack_differs_from_interp_on_variable_velocity():
    """The option reaches the kernels: on a variable velocity the two
    interface values differ (by the truncation error), on the GPU as in the
    oracle."""
    for w in (_case1d(n=4, K=8), _case2d(4, 3, 5)):
        announce(f"{w.dim}d backtrack vs interp")
        gi, _, _ = run_gpu(w)
        gb, _, _ = run_gpu(w, iface=BT)
        oi, _ = run_oracle(w)
        ob, _ = run_oracle(w, iface=BT)
        d_gpu, d_ora = rel_l2(gb, gi), rel_l2(ob, oi)
        assert d_gpu > 1e-6 and abs(d_gpu - d_ora) <= 1e-6 * d_ora


def test_backtrack_rejected_on_mixed_order_mesh():
    import paper_1910_06476_amd as P
    wm = W.c4(kx=4, nsteps=1)
    announce("mixed backtrack rejected")
    m = P.from_mixed_workload(wm)
    try:
        with pytest.raises(P.SLError):
            m.step(wm.dt, 1, iface=BT)
        m.step(wm.dt, 1)
    finally:
        m.close()
