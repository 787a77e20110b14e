"""GPU parity of the 2D mass and energy rows (targets by the RK balance law
with backtraced stage values, rows imposed after the boundary block; the
energy row by the paper's iteration in SOFT, by Newton's linearisation of
the same row in HARD) against the oracle through the C-ABI.

Most cases run with tol = 0 and a fixed sweep count on both sides; one runs
the paper's stop 1e-8.  Bar: relative L2 <= 1e-12 on the whole field."""
import numpy as np
import pytest

import workloads as W
from _parity import announce, assert_parity, rel_l2, run_gpu, run_oracle
from test_gpu_2d import _swirl_case

pytestmark = pytest.mark.gpu
TOL = 1e-12
B, M, E = W.BOUNDARY, W.MASS, W.ENERGY


@pytest.fixture(scope="module", autouse=True)
def _need_gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1910_06476_amd as P
    P.lib()


def _case(**kw):
    kw.setdefault("energy_maxit", 3)
    kw.setdefault("energy_tol", 0.0)
    kw.setdefault("nsteps", 2)
    return _swirl_case(kw.pop("kx", 4), kw.pop("ky", 3), kw.pop("n", 5), **kw)


@pytest.mark.parametrize("cmask", [B | M, B | E, B | M | E])
@pytest.mark.parametrize("mode", [W.HARD, W.SOFT])
@pytest.mark.parametrize("form", [W.ADVECTIVE, W.CONSERVATIVE])
@pytest.mark.parametrize("bc", [W.PERIODIC, W.GHOST, W.PERIODIC_X, W.PERIODIC_Y])
def test_mass_energy_matrix_parity(cmask, mode, form, bc):
    w = _case(cmask=cmask, mode=mode, form=form, bc=bc)
    announce(f"2d me cmask={cmask} mode={mode} form={form} bc={bc}")
    g, st, rc = run_gpu(w)
    o, ost = run_oracle(w)
    assert rc == 0 and (st.flags & ~2) == 0, (rc, st.flags)
    assert_parity(w, g, o)
    if cmask & E:
        assert st.max_picard == w.energy_maxit == ost.max_picard


@pytest.mark.parametrize("cmask", [M, E, M | E])
@pytest.mark.parametrize("mode", [W.HARD, W.SOFT])
def test_without_boundary_rows_parity(cmask, mode):
    w = _case(cmask=cmask, mode=mode, bc=W.GHOST)
    announce(f"2d me no boundary cmask={cmask} mode={mode}")
    g, st, rc = run_gpu(w)
    o, ost = run_oracle(w)
    assert rc == 0
    assert_parity(w, g, o)


@pytest.mark.parametrize("n", list(range(2, 17)))
def test_orders_parity(n):
    # HARD needs (n-2)^2 >= 2 free directions after the boundary block
    mode = W.HARD if (n - 2) ** 2 >= 2 else W.SOFT
    w = _case(n=n, cmask=B | M | E, mode=mode, bc=W.GHOST, nsteps=1, energy_maxit=2)
    announce(f"2d me n={n}")
    g, st, rc = run_gpu(w)
    o, ost = run_oracle(w)
    assert_parity(w, g, o)


def _swirl_divergence(w, seed=0):
    """The exact divergence u_x + v_y of _swirl_case's velocity (same seed)."""
    ph = np.random.default_rng(seed).uniform(0, 2 * np.pi, 4)
    x, y = w.coords()
    d = -0.2 * np.pi * np.sin(2 * np.pi * x + ph[1]) + 0.2 * np.pi * np.cos(2 * np.pi * y + ph[3])
    return np.ascontiguousarray(d, dtype=np.float64).ravel()


@pytest.mark.parametrize("flow", ["rotation", "swirl"])
@pytest.mark.parametrize("form", [W.ADVECTIVE, W.CONSERVATIVE])
def test_exact_divergence_parity(flow, form):
    """The divergence handed in with the velocity, on both sides: zero for
    the rotating flow (no volume terms at any node), the exact one for the
    swirl (volume terms at every node)."""
    if flow == "rotation":
        w = W.c3(kx=6, n=9, nsteps=2)
        w.cmask, w.form, w.energy_maxit, w.energy_tol = B | M | E, form, 3, 0.0
        div = w.velocity()[1]
        assert not div.any()
    else:
        w = _case(kx=5, ky=4, n=7, cmask=B | M | E, form=form, bc=W.GHOST)
        div = _swirl_divergence(w)
    announce(f"2d me exact divergence {flow} form={form}")
    g, st, rc = run_gpu(w, div=div)
    o, ost = run_oracle(w, div=div)
    assert rc == 0
    assert_parity(w, g, o)


@pytest.mark.parametrize("kx,ky", [(1, 1), (2, 1), (3, 2), (7, 5)])
def test_ragged_meshes_parity(kx, ky):
    w = _case(kx=kx, ky=ky, n=6, cmask=B | M | E, mode=W.SOFT, form=W.CONSERVATIVE)
    announce(f"2d me mesh {kx}x{ky}")
    g, st, rc = run_gpu(w)
    o, ost = run_oracle(w)
    assert_parity(w, g, o)


@pytest.mark.parametrize("rk", [1, 2, 3])
def test_rk_orders_parity(rk):
    w = _case(rk=rk, cmask=B | M, form=W.ADVECTIVE, bc=W.GHOST)
    announce(f"2d me rk={rk}")
    g, st, rc = run_gpu(w)
    o, ost = run_oracle(w)
    assert_parity(w, g, o)


def test_residuals_and_picard_statistics():
    """HARD rows hold to rounding; the statistics name the residuals and the
    Picard count."""
    w = _case(cmask=B | M | E, mode=W.HARD, energy_maxit=4)
    announce("2d me statistics")
    g, st, rc = run_gpu(w)
    o, ost = run_oracle(w)
    assert rc == 0
    assert st.max_picard == 4
    # the mass row holds to rounding; the energy row (deviation form) to
    # what the converged sweeps leave, as in the oracle
    assert st.resid_mass <= 1e-13, st.resid_mass
    # the corner values of two edges need not agree, so the boundary rows
    # hold in the least-squares sense: the residual is the oracle's
    assert abs(st.resid_boundary - ost.resid_boundary) <= 1e-12 * max(1.0, ost.resid_boundary)
    assert abs(st.resid_mass - ost.resid_mass) <= 1e-13
    assert abs(st.resid_energy - ost.resid_energy) <= 1e-9 * ost.resid_energy + 1e-15, (st.resid_energy,
                                                                                      ost.resid_energy)


@pytest.mark.parametrize("mode", [W.HARD, W.SOFT])
def test_energy_with_tolerance(mode):
    """tol > 0 (the paper's 1e-8): both sides stop by the same rule after the
    same number of sweeps, with no flag, and the fields agree."""
    w = _case(cmask=B | M | E, mode=mode, energy_maxit=50, energy_tol=1e-8, nsteps=2)
    announce(f"2d me energy tol mode={mode}")
    g, st, rc = run_gpu(w)
    o, ost = run_oracle(w)
    assert st.max_picard == ost.max_picard
    assert st.flags == ost.flags == 0
    assert_parity(w, g, o)


def test_global_mass_telescopes_on_gpu():
    """Conservative form, periodic: the face fluxes cancel between
    neighbours and the mass target has no volume term, so with a HARD mass
    row the total mass is unchanged step to step (to rounding)."""
    import paper_1910_06476_amd as P
    w = _case(kx=6, ky=5, n=6, cmask=B | M, mode=W.HARD, form=W.CONSERVATIVE, bc=W.PERIODIC, nsteps=6)
    announce("2d me telescoping")
    g, st, rc = run_gpu(w)
    xi, wq = P.sl_node_coords(w.family, w.n)
    Wr = np.outer(wq, wq).ravel() * w.dx * w.dy
    m0 = (np.asarray(w.initial()).reshape(w.K, w.nd) * Wr).sum()
    m1 = (np.asarray(g).reshape(w.K, w.nd) * Wr).sum()
    assert abs(m1 - m0) <= 1e-13 * max(1.0, abs(m0)), (m0, m1)


def test_full_size_c3_with_mass_sampled():
    """C3 shape (256x256, n=9) with boundary and mass rows, one step, in the
    launch configuration of the boundary-only bench: sampled elements
    against the oracle computed for those elements only."""
    w = W.c3(nsteps=1)
    w.cmask = B | M
    announce("c3 full size + mass, sampled")
    g, st, rc = run_gpu(w)
    rng = np.random.default_rng(5)
    elems = np.unique(np.concatenate([rng.choice(w.K, 48, replace=False), [0, 255, w.K - 256, w.K - 1]]))
    want = np.zeros(w.K, dtype=np.uint8)
    want[elems] = 1
    o, ost = run_oracle(w, want=want)
    assert rc == 0
    assert_parity(w, g, o, elems=elems)


@pytest.mark.parametrize("cmask", [B | M, B | M | E])
def test_full_size_c3_bench_options_sampled(cmask):
    """The options `bench.py --workload c3 --constraints bm` / `bme` times:
    full C3 size, the flow's exact divergence (zero) handed to both sides,
    HARD, the energy stop 1e-8 with up to 50 sweeps; one step, sampled
    elements against the oracle computed for those elements only."""
    w = W.c3(nsteps=1)
    w.cmask = cmask
    div = w.velocity()[1]
    announce(f"c3 full size, bench options cmask={cmask}, sampled")
    g, st, rc = run_gpu(w, div=div)
    rng = np.random.default_rng(11)
    elems = np.unique(np.concatenate([rng.choice(w.K, 48, replace=False), [0, 255, w.K - 256, w.K - 1]]))
    want = np.zeros(w.K, dtype=np.uint8)
    want[elems] = 1
    o, ost = run_oracle(w, want=want, div=div)
    assert rc == 0 and st.flags == 0, (rc, st.flags)
    assert_parity(w, g, o, elems=elems)


@pytest.mark.parametrize("n,cmask,ok", [(2, B | M, False), (3, B | M, True), (3, B | M | E, False),
                                        (4, B | M | E, True)])
def test_hard_rows_beyond_boundary_null_space_rejected(n, cmask, ok):
    """null(C_B) has dimension (n-2)^2: sl_step refuses more HARD rows than
    that, before any launch; SOFT accepts them."""
    import paper_1910_06476_amd as P
    w = _case(n=n, cmask=cmask, mode=W.HARD, nsteps=1)
    announce(f"2d hard rows n={n} cmask={cmask}")
    if ok:
        g, st, rc = run_gpu(w)
        assert rc == 0
    else:
        with pytest.raises(P.SLError) as e:
            run_gpu(w)
        assert e.value.status == P.SL_E_INVALID
    g, st, rc = run_gpu(w, mode=W.SOFT)
    assert rc == 0
