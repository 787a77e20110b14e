"""GPU parity of the 1D HIP path against the oracle, through the C-ABI, on
seeded synthetic inputs from ``workloads``.

Bar: relative L2 <= 1e-12 (FP64) on the whole field, every case, with the
energy row included (it is solved in the deviation form on both sides, so
its result is as well conditioned as the rest)."""
import numpy as np
import pytest

import workloads as W
from _parity import announce, assert_parity, opts_dict, rel_l2, run_gpu, run_oracle

pytestmark = pytest.mark.gpu
TOL = 1e-12


@pytest.fixture(scope="module", autouse=True)
def _need_gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1910_06476_amd as P
    P.lib()


def _random_state(w, seed):
    return W.random_field_1d(w.K, w.n, seed, family=w.family, x0=w.x0, x1=w.x1)


def test_c1_one_step_parity():
    w = W.c1()
    for phi0 in (w.initial(), _random_state(w, 1)):
        announce("c1 one step")
        g, st, rc = run_gpu(w, phi0=phi0, nsteps=1)
        o, ost = run_oracle(w, phi0=phi0, nsteps=1)
        assert rc == 0 and st.flags == 0
        assert rel_l2(g, o) <= TOL


def test_c1_full_run_parity_and_accuracy():
    w = W.c1()
    announce("c1 200 steps")
    g, st, rc = run_gpu(w)
    o, ost = run_oracle(w)
    assert rc == 0
    assert rel_l2(g, o) <= TOL
    assert w.l2_error(g, w.nsteps * w.dt) < 5e-8


def _case(n=7, K=37, rk=4, cmask=W.BOUNDARY, mode=W.HARD, form=W.ADVECTIVE, bc=W.PERIODIC, seed=0):
    x0, x1 = 0.0, 1.0
    rng = np.random.default_rng(seed)
    ph = rng.uniform(0.2, 0.5)
    dt = 0.2 * W.min_gap(W.GL, n) * (x1 - x0) / K / 0.95
    w = W.Workload(name="case", dim=1, kx=K, ky=1, n=n, family=W.GL, x0=x0, x1=x1, y0=0, y1=1, bc=bc,
                   form=form, rk=rk, cmask=cmask, mode=mode, dt=dt, nsteps=3,
                   u0=lambda xx, yy: 1.2 + np.sin(2 * np.pi * xx) + 0.3 * np.cos(6 * np.pi * xx + ph),
                   vel=lambda xx, yy: (0.7 + 0.25 * np.sin(2 * np.pi * xx + ph), 0.0, 0.0),
                   exact=lambda xx, yy, t: 1.2 + np.sin(2 * np.pi * (xx - 0.7 * t)),
                   energy_tol=0.0, energy_maxit=3)
    return w


@pytest.mark.parametrize("bc", [W.PERIODIC, W.GHOST])
@pytest.mark.parametrize("form", [W.ADVECTIVE, W.CONSERVATIVE])
@pytest.mark.parametrize("mode", [W.HARD, W.SOFT])
@pytest.mark.parametrize("cmask", [W.BOUNDARY, W.BOUNDARY | W.MASS, W.BOUNDARY | W.MASS | W.ENERGY, W.MASS])
@pytest.mark.parametrize("rk", [1, 2, 3, 4])
def test_option_matrix_parity(rk, cmask, mode, form, bc):
    w = _case(rk=rk, cmask=cmask, mode=mode, form=form, bc=bc)
    announce(f"matrix rk={rk} cmask={cmask} mode={mode} form={form} bc={bc}")
    g, st, rc = run_gpu(w)
    o, ost = run_oracle(w)
    assert_parity(w, g, o)
    assert st.max_picard == ost.max_picard
    assert st.flags == ost.flags


@pytest.mark.parametrize("n", list(range(2, 18)))
def test_orders_parity(n):
    cmask = W.BOUNDARY | W.MASS | W.ENERGY if n >= 4 else W.BOUNDARY
    w = _case(n=n, K=53, cmask=cmask)
    announce(f"order n={n}")
    g, st, rc = run_gpu(w)
    o, ost = run_oracle(w)
    assert_parity(w, g, o)


@pytest.mark.parametrize("K", [1, 2, 3, 14, 15, 16, 31, 47, 301])
@pytest.mark.parametrize("bc", [W.PERIODIC, W.GHOST])
def test_ragged_sizes_parity(K, bc):
    """K around the 14 elements a 256-lane advect block holds at n=17 (18
    lanes each) and the 32 a constrain wave holds, and a few larger ragged
    counts."""
    w = _case(n=17, K=K, bc=bc, cmask=W.BOUNDARY | W.MASS | W.ENERGY)
    announce(f"ragged K={K} bc={bc}")
    g, st, rc = run_gpu(w)
    o, ost = run_oracle(w)
    assert_parity(w, g, o)


def test_chebyshev_nodes_paper_problem_parity():
    """The paper's section 5.2 problem (conservative, Chebyshev-Gauss nodes,
    H=4, P=6) with all constraints in SOFT mode, a few steps."""
    w = W.x6(rk=2, cmask=W.BOUNDARY | W.MASS | W.ENERGY)
    w.energy_tol = 0.0
    w.energy_maxit = 4
    announce("x6 soft")
    g, st, rc = run_gpu(w, nsteps=8)
    o, ost = run_oracle(w, nsteps=8)
    assert rel_l2(g, o) <= TOL, rel_l2(g, o)


def test_paper_table3_basecase1_through_the_abi():
    """Table 3 Basecase1 (section 5.2) reproduced by the HIP path itself."""
    w = W.x6(rk=1, cmask=W.BOUNDARY, mode=W.SOFT)
    announce("x6 basecase1")
    g, st, rc = run_gpu(w)
    import oracle
    xi, wq = oracle.nodes(w.family, w.n)
    x = w.x0 + (np.arange(w.K)[:, None] + xi[None, :]) * w.dx
    ex = w.exact(x, None, w.nsteps * w.dt)
    l2 = np.sqrt(((g.reshape(w.K, w.n) - ex) ** 2 * wq * w.dx).sum(1)).sum()
    assert float("%.2e" % l2) == 5.25e-2


def test_c2_shape_multistep_parity():
    w = W.c2(K=512, nsteps=20)
    w.energy_tol = 0.0
    w.energy_maxit = 2
    announce("c2 K=512 20 steps")
    g, st, rc = run_gpu(w)
    o, ost = run_oracle(w)
    assert_parity(w, g, o)
    assert st.resid_mass < 1e-15 and st.resid_boundary < 1e-13


@pytest.mark.parametrize("cmask", [W.BOUNDARY, W.BOUNDARY | W.MASS, W.BOUNDARY | W.MASS | W.ENERGY])
def test_c2_full_size_parity(cmask):
    """Full size (K=65536, n=17, RK4) in the launch configuration the
    benchmark times, one step, compared on the whole field (the oracle takes
    about a second).  Picard runs exactly one sweep on both sides."""
    w = W.c2(cmask=cmask)
    announce(f"c2 full size one step cmask={cmask}")
    g, st, rc = run_gpu(w, nsteps=1, energy_tol=0.0, energy_maxit=1)
    o, ost = run_oracle(w, nsteps=1, energy_tol=0.0, energy_maxit=1)
    assert_parity(w, g, o)
    assert rc == 0 and st.flags == 0


def test_c2_probe_size_parity():
    """The HBM probe's size (K=2^22, n=17, RK4, boundary rows) in the launch
    configuration the benchmark times, one step, compared on the whole field
    (71.3 M values; the oracle takes a few seconds on the host's cores)."""
    w = W.c2(K=1 << 22, cmask=W.BOUNDARY)
    announce("c2 probe size K=2^22 one step")
    g, st, rc = run_gpu(w, nsteps=1)
    o, ost = run_oracle(w, nsteps=1)
    assert_parity(w, g, o)
    assert rc == 0 and st.flags == 0


def test_c2_benchmark_options_parity():
    """Full C2 in exactly the benchmark's options (K=65536, n=17, RK4,
    boundary + mass + energy HARD, the paper's stop 1e-8, cap 50), three
    steps: whole-field parity, the same flags (none) and the same largest
    sweep count on both sides, and the error against the closed form at the
    level of boundary + mass alone."""
    w = W.c2(nsteps=3)
    assert (w.cmask, w.mode, w.rk, w.energy_tol, w.energy_maxit) == (
        W.BOUNDARY | W.MASS | W.ENERGY, W.HARD, 4, 1e-8, 50)
    announce("c2 full size 3 steps, benchmark options")
    g, st, rc = run_gpu(w)
    o, ost = run_oracle(w)
    err = assert_parity(w, g, o)
    assert rc == 0 and st.flags == 0 and ost.flags == 0
    assert st.max_picard == ost.max_picard
    assert st.resid_boundary < 1e-12 and st.resid_mass < 1e-16
    assert w.l2_error(g, w.nsteps * w.dt) < 1e-13
    print(f"c2 benchmark options: rel L2 vs oracle {err:.2e}, sweeps {st.max_picard}")


def test_bitwise_determinism():
    w = _case(n=17, K=301, cmask=W.BOUNDARY | W.MASS | W.ENERGY)
    announce("determinism")
    g1, _, _ = run_gpu(w)
    g2, _, _ = run_gpu(w)
    assert np.array_equal(g1, g2)


def test_error_paths_on_device():
    import paper_1910_06476_amd as P
    w = W.c1()
    announce("errors")
    m = P.Mesh(1, w.kx, 1, w.n - 1, w.initial(), x0=w.x0, x1=w.x1)
    try:
        with pytest.raises(P.SLError) as e:
            m.step(w.dt)
        assert e.value.status == P.SL_E_STATE
        a, _ = w.velocity()
        bad = a.copy()
        bad[3] = np.nan
        with pytest.raises(P.SLError) as e:
            m.set_velocity(bad)
        assert e.value.status == P.SL_E_NONFINITE
        m.set_velocity(a)
        with pytest.raises(P.SLError) as e:
            m.step(m.max_dt(1.0) * 1.01)
        assert e.value.status == P.SL_E_CFL
        with pytest.raises(P.SLError) as e:
            m.set_ghost(np.zeros(2))
        assert e.value.status == P.SL_E_STATE
        m.step(m.max_dt(0.5), 2)
        rc, out, st = m.read()
        assert rc == 0 and st.steps == 2
        # the paper's restriction admits equality: the particle next to the
        # edge lands on it, inside the containment tolerance
        m.step(m.max_dt(1.0), 1)
        rc, out, st = m.read()
        assert rc == 0 and st.flags == 0 and np.all(np.isfinite(out))
    finally:
        m.close()


@pytest.mark.parametrize("form", [W.ADVECTIVE, W.CONSERVATIVE])
@pytest.mark.parametrize("rk", [1, 2, 3, 4])
def test_linear_velocity_closed_form(rk, form):
    """The device step against mathematics, not only the oracle: for a = c x
    (2D: (c x, c y)) and a linear field, one step without constraint rows is
    u0 / R(c dt) (advective) or R(-d c dt) / R(c dt) u0 (conservative), R the
    degree-rk Taylor polynomial of e^z (tests/_linear_flow.py); the
    next-order polynomial would differ by more than 1e-10."""
    import _linear_flow as LF
    w, a, div, ghost, expect = LF.case(1, rk, form)
    announce(f"linear velocity 1D rk={rk} form={form}")
    g, st, rc = run_gpu(w, nsteps=1, ghost=ghost)
    assert rc == 0 and st.flags == 0
    np.testing.assert_allclose(g, expect, rtol=0, atol=1e-14)


@pytest.mark.parametrize("nsteps", [2, 5, 6])
def test_multistep_call_equals_single_steps(nsteps):
    """Several steps in one sl_step call (counts odd and even, so a call can
    start from either ping-pong buffer) equal one sl_step per step: the
    field and the statistics, bit for bit."""
    import paper_1910_06476_amd as P
    w = W.c2(K=301, nsteps=nsteps)
    announce(f"1d multistep vs single steps nsteps={nsteps}")
    opts = opts_dict(w)
    calls = [nsteps, 3, 4, 2]
    mg = P.from_workload(w)
    me = P.from_workload(w)
    try:
        for c in calls:
            mg.step(w.dt, c, **opts)
            for _ in range(c):
                me.step(w.dt, 1, **opts)
        rg, g, sg = mg.read()
        re_, e, se = me.read()
    finally:
        mg.close()
        me.close()
    assert np.array_equal(g, e)
    assert (rg, sg.steps, sg.flags, sg.max_picard) == (re_, se.steps, se.flags, se.max_picard)
    assert sg.steps == sum(calls)


@pytest.mark.parametrize("dim", [1, 2])
def test_zero_steps_leave_the_field(dim):
    """sl_step with nsteps = 0 launches nothing: the field reads back as
    given, bit for bit, with no steps counted and no flags; a negative count
    is rejected."""
    import paper_1910_06476_amd as P
    w = W.c2(K=40) if dim == 1 else W.c3(kx=5, n=6)
    announce(f"zero steps {dim}D")
    m = P.from_workload(w)
    try:
        if w.bc != W.PERIODIC:
            m.set_ghost(w.ghost_rows(0.0, 2))
        m.step(w.dt, 0, **opts_dict(w))
        rc, out, st = m.read()
        assert rc == 0 and st.steps == 0 and st.flags == 0
        assert np.array_equal(out, w.initial())
        with pytest.raises(P.SLError) as e:
            m.step(w.dt, -1, **opts_dict(w))
        assert e.value.status == P.SL_E_INVALID
    finally:
        m.close()


@pytest.mark.parametrize("mode", [W.HARD, W.SOFT])
@pytest.mark.parametrize("cmask", [W.BOUNDARY, W.BOUNDARY | W.MASS | W.ENERGY])
def test_zero_velocity(cmask, mode):
    """a = 0, every face on the zero-speed tie rule (tests/_zerovel.py): a
    global polynomial comes back unchanged on the device; a periodic field
    whose element traces differ matches the oracle."""
    import _zerovel
    w = _zerovel.polynomial_case(1, cmask, mode)
    announce(f"zero velocity 1D cmask={cmask} mode={mode}")
    g, st, rc = run_gpu(w)
    assert rc == 0 and st.flags == 0
    np.testing.assert_allclose(g, w.initial(), rtol=0, atol=1e-13)
    w = _zerovel.periodic_case(1, cmask, mode)
    g, st, rc = run_gpu(w)
    o, ost = run_oracle(w)
    assert rc == 0
    assert_parity(w, g, o)
