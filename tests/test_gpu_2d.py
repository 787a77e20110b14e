"""GPU parity of the 2D HIP path (eq. 5.1, 5.4, 2dx/2dy_bnd_interpolate,
boundary least squares) against the oracle through the C-ABI.

The oracle solves the moved-point Vandermonde system of eq. 5.4 by LU with
partial pivoting; the HIP path by matrix-free defect correction with a
separable preconditioner, so agreement to 1e-12 is a check of the solver as
well.  Bar: relative L2 <= 1e-12 (FP64)."""
import math

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


def _swirl_case(kx, ky, n, bc=W.PERIODIC, form=W.ADVECTIVE, mode=W.HARD, rk=4, nsteps=3, family=W.GL, seed=0,
                cmask=W.BOUNDARY, energy_maxit=50, energy_tol=1e-8):
    """Seeded smooth velocity with nonzero divergence and a random-mode field."""
    rng = np.random.default_rng(seed)
    ph = rng.uniform(0, 2 * math.pi, 4)
    u = lambda x, y: 0.6 + 0.3 * np.sin(2 * math.pi * y + ph[0]) + 0.1 * np.cos(2 * math.pi * x + ph[1])
    v = lambda x, y: -0.4 + 0.25 * np.cos(2 * math.pi * x + ph[2]) + 0.1 * np.sin(2 * math.pi * y + ph[3])
    f0 = lambda x, y: 1.3 + np.sin(2 * math.pi * x) * np.cos(2 * math.pi * y + 0.3) + 0.2 * np.cos(4 * math.pi * x)
    amax = 1.0
    dt = 0.2 * W.min_gap(family, n) * min(1.0 / kx, 1.0 / ky) / amax
    return W.Workload(name="swirl2", dim=2, kx=kx, ky=ky, n=n, family=family, x0=0.0, x1=1.0, y0=0.0, y1=1.0,
                      bc=bc, form=form, rk=rk, cmask=cmask, mode=mode, dt=dt, nsteps=nsteps,
                      energy_maxit=energy_maxit, energy_tol=energy_tol,
                      u0=f0, vel=lambda x, y: (u(x, y), v(x, y), 0.0),
                      exact=lambda x, y, t: f0(x - 0.6 * t, y + 0.4 * t))


@pytest.mark.parametrize("n", [3, 6, 9, 11])
@pytest.mark.parametrize("mode", [W.HARD, W.SOFT])
def test_fp32_refined_remap_parity(n, mode):
    """SL_PREC_FP32_REFINED: FP32 preconditioner, FP64 residual and iterate.
    Defect correction converges to the same FP64 solution of eq. 5.4, so the
    FP64 bar holds."""
    w = _swirl_case(4, 5, n, mode=mode, form=W.CONSERVATIVE, nsteps=4)
    announce(f"2d fp32-refined n={n} mode={mode}")
    g, st, rc = run_gpu(w, precision=1)
    o, ost = run_oracle(w)
    assert rc == 0 and (st.flags & ~2) == 0, st.flags
    assert rel_l2(g, o) <= TOL, rel_l2(g, o)


def test_fp32_refined_tiny_values():
    """The hill's tail reaches 1e-33, so residuals of the remap solve fall
    below the FP32 normal range unless the preconditioner's operand is
    rescaled; every element must still converge."""
    w = W.c3(kx=8, nsteps=5)
    announce("c3 8x8 fp32-refined")
    g, st, rc = run_gpu(w, precision=1)
    o, ost = run_oracle(w)
    assert rc == 0 and st.flags == 0, (rc, st.flags)
    assert st.remap_sweeps_max < 60
    assert rel_l2(g, o) <= TOL, rel_l2(g, o)


@pytest.mark.parametrize("n", [3, 6, 9, 11])
@pytest.mark.parametrize("mode", [W.HARD, W.SOFT])
def test_bf16_refined_remap_parity(n, mode):
    """SL_PREC_BF16_REFINED: BF16 preconditioner entries and operands, FP32
    sums, FP64 residual and iterate.  Each sweep contracts the error only to
    about the BF16 rounding (2^-9) times the preconditioner's size, so more
    sweeps are needed, but the limit is the same FP64 solution of eq. 5.4."""
    w = _swirl_case(4, 5, n, mode=mode, form=W.CONSERVATIVE, nsteps=4)
    announce(f"2d bf16-refined n={n} mode={mode}")
    g, st, rc = run_gpu(w, precision=2)
    o, ost = run_oracle(w)
    assert rc == 0 and (st.flags & ~2) == 0, st.flags
    assert rel_l2(g, o) <= TOL, rel_l2(g, o)


def test_bf16_refined_tiny_values_and_sweeps():
    """The hill's tail (1e-33) with BF16 operands: the power-of-two scaling
    keeps them in the normal range; every element converges within the cap,
    in more sweeps than the FP32 and FP64 preconditioners need."""
    w = W.c3(kx=8, nsteps=5)
    announce("c3 8x8 bf16-refined")
    g, st, rc = run_gpu(w, precision=2)
    _, s32, _ = run_gpu(w, precision=1)
    _, s64, _ = run_gpu(w)
    o, ost = run_oracle(w)
    assert rc == 0 and st.flags == 0, (rc, st.flags)
    assert st.remap_sweeps_max < 60
    assert st.remap_sweeps_mean > s32.remap_sweeps_mean >= s64.remap_sweeps_mean
    assert rel_l2(g, o) <= TOL, rel_l2(g, o)


def test_c3_shape_small_parity():
    w = W.c3(kx=8, nsteps=10)
    announce("c3 8x8 10 steps")
    g, st, rc = run_gpu(w)
    o, ost = run_oracle(w)
    assert rc == 0 and st.flags == 0
    assert rel_l2(g, o) <= TOL, rel_l2(g, o)


@pytest.mark.parametrize("mode", [W.HARD, W.SOFT])
@pytest.mark.parametrize("form", [W.ADVECTIVE, W.CONSERVATIVE])
@pytest.mark.parametrize("bc", [W.PERIODIC, W.GHOST, W.PERIODIC_X, W.PERIODIC_Y])
def test_swirl_matrix_parity(mode, form, bc):
    w = _swirl_case(5, 7, 6, bc=bc, form=form, mode=mode)
    announce(f"swirl mode={mode} form={form} bc={bc}")
    g, st, rc = run_gpu(w)
    o, ost = run_oracle(w)
    assert rel_l2(g, o) <= TOL, rel_l2(g, o)
    assert (st.flags & ~2) == 0


@pytest.mark.parametrize("rk", [1, 2, 3, 4])
def test_rk_orders_parity(rk):
    w = _swirl_case(4, 3, 5, rk=rk, form=W.CONSERVATIVE)
    announce(f"2d rk={rk}")
    g, st, rc = run_gpu(w)
    o, ost = run_oracle(w)
    assert rel_l2(g, o) <= TOL, rel_l2(g, o)


@pytest.mark.parametrize("n", list(range(2, 18)))
def test_orders_parity(n):
    w = _swirl_case(4, 5, n, bc=W.GHOST)
    announce(f"2d n={n}")
    g, st, rc = run_gpu(w)
    o, ost = run_oracle(w)
    assert rel_l2(g, o) <= TOL, rel_l2(g, o)


@pytest.mark.parametrize("mode", [W.HARD, W.SOFT])
@pytest.mark.parametrize("bc", [W.PERIODIC, W.PERIODIC_X])
def test_order_16_parity(bc, mode):
    """17 nodes per direction (289 particles): one element per 320-lane
    block in the advect, two nodes per lane in the boundary-row solve."""
    w = _swirl_case(3, 2, 17, bc=bc, mode=mode, form=W.CONSERVATIVE)
    announce(f"2d n=17 bc={bc} mode={mode}")
    g, st, rc = run_gpu(w)
    o, ost = run_oracle(w)
    assert rc == 0
    assert rel_l2(g, o) <= TOL, rel_l2(g, o)


def test_order_16_refuses_what_it_does_not_run():
    """Order 16 in 2D: FP64 with boundary rows only; the rest is refused
    before any launch."""
    import paper_1910_06476_amd as P
    w = _swirl_case(2, 2, 17, bc=W.PERIODIC)
    with pytest.raises(P.SLError):
        P.Mesh(2, 2, 2, 16, w.initial(), precision=P.SL_PREC_FP32_REFINED)
    m = P.from_workload(w)
    try:
        with pytest.raises(P.SLError):
            m.step(w.dt, 1, rk=4, constraints=W.BOUNDARY | W.MASS, mode=W.HARD)
        m.step(w.dt, 1, rk=4, constraints=W.BOUNDARY, mode=W.HARD)
        rc, out, st = m.read()
        assert rc == 0 and st.steps == 1
    finally:
        m.close()


@pytest.mark.parametrize("kx,ky", [(1, 1), (1, 2), (2, 1), (3, 1), (2, 2), (5, 7), (11, 3)])
def test_ragged_meshes_parity(kx, ky):
    """E = 3 elements per block at n = 9: sizes around the block packing,
    single-element periodic meshes (an element is its own neighbour)."""
    w = _swirl_case(kx, ky, 9)
    announce(f"2d mesh {kx}x{ky}")
    g, st, rc = run_gpu(w)
    o, ost = run_oracle(w)
    assert rel_l2(g, o) <= TOL, rel_l2(g, o)


def test_paper_2d_constant_velocity_parity():
    """Section 5.3 (a=2, b=1, sin 2pi x sin 2pi y, periodic), Chebyshev-Gauss
    nodes, SOFT (the paper's least squares), H=4, P=6, a few steps."""
    w = W.x9(P=6, H=4, rk=1)
    announce("x9")
    g, st, rc = run_gpu(w, nsteps=5)
    o, ost = run_oracle(w, nsteps=5)
    assert rel_l2(g, o) <= TOL, rel_l2(g, o)


def test_c3_full_size_sampled_parity():
    """Full C3 size (256x256, n=9, rotation, ghost inflow), one step in the
    benchmarked launch configuration; the oracle computes a seeded sample of
    elements (with their neighbours)."""
    w = W.c3()
    rng = np.random.default_rng(0)
    sample = np.unique(np.concatenate([[0, 1, 2, 255, 256, w.K - 1, w.K - 256],
                                       rng.integers(0, w.K, 120)]))
    want = np.zeros(w.K, dtype=np.uint8)
    want[sample] = 1
    announce("c3 full size one step")
    g, st, rc = run_gpu(w, nsteps=1)
    o, ost = run_oracle(w, nsteps=1, want=want)
    G = g.reshape(w.K, w.nd)[sample]
    O = o.reshape(w.K, w.nd)[sample]
    assert rc == 0 and st.flags == 0
    assert rel_l2(G, O) <= TOL, rel_l2(G, O)


def test_c3_full_size_accuracy_after_steps():
    """50 steps of the rotating hill at full size: no flags, and the L2 error
    against the rotated exact solution stays at the interpolation level."""
    w = W.c3(nsteps=50)
    announce("c3 full size 50 steps")
    g, st, rc = run_gpu(w)
    assert rc == 0 and st.flags == 0
    err = w.l2_error(g, w.nsteps * w.dt)
    assert err < 1e-6, err


def test_2d_bitwise_determinism():
    w = _swirl_case(5, 7, 9, form=W.CONSERVATIVE)
    announce("2d determinism")
    g1, _, _ = run_gpu(w)
    g2, _, _ = run_gpu(w)
    assert np.array_equal(g1, g2)


def test_remap_solve_statistics():
    """The iterative remap solve reports its sweeps and last relative
    correction; a converged solve stops at or below 2^-44."""
    import paper_1910_06476_amd as P
    w = _swirl_case(6, 6, 9, nsteps=4)
    m = P.from_workload(w)
    try:
        m.step(w.dt, 4, rk=4, constraints=W.BOUNDARY, mode=W.HARD)
        rc, _, st = m.read()
        assert rc == 0
        assert 1 <= st.remap_sweeps_max <= 60
        assert 1.0 <= st.remap_sweeps_mean <= st.remap_sweeps_max
        assert 0.0 <= st.refine_resid <= 2.0 ** -44
        rc, _, st = m.read()  # nothing stepped since the last read
        assert st.remap_sweeps_mean == 0.0 and st.remap_sweeps_max == 0
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
    w, a, div, ghost, expect = LF.case(2, rk, form)
    announce(f"linear velocity 2D rk={rk} form={form}")
    g, st, rc = run_gpu(w, nsteps=1, ghost=ghost)
    assert rc == 0 and st.flags == 0
    np.testing.assert_allclose(g, expect, rtol=0, atol=1e-13)


@pytest.mark.parametrize("mode", [W.HARD, W.SOFT])
@pytest.mark.parametrize("bc", [W.PERIODIC_X, W.PERIODIC_Y])
@pytest.mark.parametrize("deg,cmask", [(4, W.BOUNDARY), (1, W.BOUNDARY | W.MASS | W.ENERGY)])
def test_periodic_in_one_direction(bc, deg, cmask, mode):
    """Periodic in one direction, ghost values on the sides of the other
    (tests/_onedir.py): a polynomial across the ghost sides moved by a
    constant velocity is reproduced exactly on the device, equal to the
    oracle, and the NaN ghost values of the periodic sides are never read."""
    import _onedir
    w, g = _onedir.case(bc, deg, cmask, mode)
    announce(f"one-direction periodic bc={bc} deg={deg} cmask={cmask} mode={mode}")
    gp, st, rc = run_gpu(w, ghost=g)
    o, ost = run_oracle(w, ghost=g)
    assert rc == 0 and st.flags == 0 and np.all(np.isfinite(gp))
    assert_parity(w, gp, o)
    ex = w.exact_at(w.nsteps * w.dt)
    np.testing.assert_allclose(gp, ex, rtol=0, atol=1e-11 * max(1.0, np.abs(ex).max()))


@pytest.mark.parametrize("nsteps", [2, 5])
def test_multistep_call_equals_single_steps(nsteps):
    """2D periodic mesh with mass and energy rows: several steps in one
    sl_step call equal one sl_step per step, bit for bit."""
    import paper_1910_06476_amd as P
    w = _swirl_case(5, 4, 6, nsteps=nsteps, cmask=W.BOUNDARY | W.MASS | W.ENERGY, energy_tol=0.0, energy_maxit=3)
    announce(f"2d multistep vs single steps nsteps={nsteps}")
    opts = opts_dict(w)
    calls = [nsteps, 3, 2]
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


@pytest.mark.parametrize("mode", [W.HARD, W.SOFT])
@pytest.mark.parametrize("cmask", [W.BOUNDARY, W.BOUNDARY | W.MASS | W.ENERGY])
def test_zero_velocity(cmask, mode):
    """a = 0, every face on the zero-speed tie rule (tests/_zerovel.py): a
    global polynomial comes back unchanged on the device; a periodic field
    whose element traces differ matches the oracle."""
    import _zerovel
    w = _zerovel.polynomial_case(2, cmask, mode)
    announce(f"zero velocity 2D cmask={cmask} mode={mode}")
    g, st, rc = run_gpu(w)
    assert rc == 0 and st.flags == 0
    np.testing.assert_allclose(g, w.initial(), rtol=0, atol=1e-13)
    w = _zerovel.periodic_case(2, cmask, mode)
    g, st, rc = run_gpu(w)
    o, ost = run_oracle(w)
    assert rc == 0
    assert_parity(w, g, o)
