"""The paper's own test suite run by the HIP path through the C-ABI.

* Table 3 (section 5.2, phi_t + (-sin(x) phi)_x = 0, H = 4, P = 6, T = 1):
  the pinned rows Basecase1, Basecase2, MF2 and MF3 reproduced by the device
  at the printed digits, and equal to the oracle.
* P-convergence with constant velocity (section 5.1, Fig. fig:1_2; H = 4,
  T = 10): Basecase converges exponentially in P, MF1 is bound by its
  first-order time integration, MF2 improves algebraically, MF3 matches
  Basecase.
* Dirichlet against periodic (section 5.1, Fig. fig:1_3): with exact inflow
  values the Basecase error is below the periodic one at every P.
* P-convergence with variable velocity (section 5.2, Fig. fig:2_2; H = 4,
  T = 1): with the explicit step the first-order schemes converge
  algebraically, the second-order ones spectrally until the time error
  bounds them, MF3 furthest; with dt = 1e-4 the first-order schemes converge
  spectrally to P = 8 and are then bound at O(1e-4), while the second-order
  one keeps converging.

The claims are the paper's; the thresholds are set from the oracle's values
under the readings listed in the design notes, with margins.  Every run
sampled here matches the oracle to 1e-12 (relative L2) over one step, and
over the whole run to 1e-15 per step of rounding drift."""
import math
import os

import numpy as np
import pytest

import workloads as W
from _parity import announce, rel_l2, run_gpu, run_oracle

pytestmark = pytest.mark.gpu
TOL = 1e-12
GOLD = os.path.join(os.path.dirname(__file__), "golden")
CASES = {"Basecase1": (1, W.BOUNDARY), "MF1": (1, W.BOUNDARY | W.MASS), "Basecase2": (2, W.BOUNDARY),
         "MF2": (2, W.BOUNDARY | W.MASS), "MF3": (3, W.BOUNDARY | W.MASS)}


@pytest.fixture(scope="module", autouse=True)
def _need_gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1910_06476_amd as P
    P.lib()


def _norms(w, phi, t):
    """The paper's L2 norm (eq. 5.2, physical dx) and the ratios of the global
    mass and energy to the exact ones."""
    import oracle
    xi, wq = oracle.nodes(w.family, w.n)
    x = w.x0 + (np.arange(w.K)[:, None] + xi[None, :]) * w.dx
    ex = w.exact(x, None, t)
    P = np.asarray(phi).reshape(w.K, w.n)
    l2 = np.sqrt(((P - ex) ** 2 * wq * w.dx).sum(1)).sum()
    return l2, (P * wq).sum() / (ex * wq).sum() - 1.0, (P ** 2 * wq).sum() / (ex ** 2 * wq).sum()


def _sig(x, like):
    mant = like.lower().split("e")[0].lstrip("-")
    digits = len(mant.replace(".", "").lstrip("0")) or 1
    if "e" in like.lower():
        return float("%.*e" % (digits - 1, x))
    dec = len(mant.split(".")[1]) if "." in mant else 0
    return round(x, dec)


def _table3_row(case):
    for line in open(os.path.join(GOLD, "table3.txt")):
        f = line.split()
        if f and f[0] == case:
            return f
    raise KeyError(case)


# Rounding drift between two FP64 implementations over a whole run grows with
# the step count: held to 1e-15 per step (1e-11 over the 10^4 steps of the
# dt = 1e-4 runs); the per-step gate stays 1e-12.
DRIFT_PER_STEP = 1e-15


def _gpu_l2(w, parity=False):
    announce(f"{w.name} P={w.n - 1} H={w.K} rk={w.rk} cmask={w.cmask} bc={w.bc} dt={w.dt:.3g} steps={w.nsteps}")
    g, st, rc = run_gpu(w)
    if parity:
        g1, _, _ = run_gpu(w, nsteps=1)
        o1, _ = run_oracle(w, nsteps=1)
        assert rel_l2(g1, o1) <= TOL, rel_l2(g1, o1)
        o, ost = run_oracle(w)
        assert rel_l2(g, o) <= max(TOL, DRIFT_PER_STEP * w.nsteps), (rel_l2(g, o), w.nsteps)
    return _norms(w, g, w.nsteps * w.dt)[0]


@pytest.mark.parametrize("case", ["Basecase1", "Basecase2", "MF2", "MF3"])
def test_table3_pinned_rows_through_the_abi(case):
    rk, cmask = {"Basecase1": (1, W.BOUNDARY), "Basecase2": (2, W.BOUNDARY),
                 "MF2": (2, W.BOUNDARY | W.MASS), "MF3": (3, W.BOUNDARY | W.MASS)}[case]
    row = _table3_row(case)
    w = W.x6(rk=rk, cmask=cmask)
    announce(f"table 3 {case}")
    g, st, rc = run_gpu(w)
    o, ost = run_oracle(w)
    assert rel_l2(g, o) <= TOL, rel_l2(g, o)
    l2, dm, e = _norms(w, g, w.nsteps * w.dt)
    assert _sig(dm, row[1]) == float(row[1]) or (float(row[1]) == 0 and abs(dm) < 5e-5), (case, dm)
    assert _sig(e, row[2]) == float(row[2]), (case, e)
    assert _sig(l2, row[3]) == float(row[3]), (case, l2)


def test_p_convergence_constant_velocity():
    """Section 5.1, Fig. fig:1_2 (H = 4, T = 10, P = 3..10)."""
    Ps = list(range(3, 11))
    err = {c: [] for c in CASES}
    for c, (rk, cmask) in CASES.items():
        for P in Ps:
            err[c].append(_gpu_l2(W.x1(P=P, H=4, rk=rk, cmask=cmask), parity=P in (4, 9)))
    b, mf1, mf2, mf3 = (np.array(err[c]) for c in ("Basecase1", "MF1", "MF2", "MF3"))
    # Basecase: exponential, a factor of more than 5 per order, 1e8 overall
    assert np.all(b[1:] < b[:-1] / 5) and b[0] / b[-1] > 1e8
    # the integrator does not matter for Basecase with constant velocity
    np.testing.assert_allclose(err["Basecase2"], b, rtol=0.05)
    # MF1: bound by the first-order time integration (less than 100x overall,
    # 1e-3 or more at P = 10)
    assert mf1[0] / mf1[-1] < 100 and mf1[-1] > 1e-3
    # MF2: algebraic once the time error dominates, far above Basecase at P = 10
    assert mf2[-1] > 1e4 * b[-1] and np.all(mf2[4:] < mf2[3:-1])
    # MF3: matches Basecase
    np.testing.assert_allclose(mf3, b, rtol=0.1)


def test_dirichlet_more_accurate_than_periodic():
    """Section 5.1, Fig. fig:1_3: Basecase with exact inflow values
    (Dirichlet) against periodic, H = 4, T = 10, P = 3..9."""
    for P in range(3, 10):
        r = []
        for bc in (W.PERIODIC, W.GHOST):
            w = W.x1(P=P, H=4, rk=1)
            w.bc = bc
            r.append(_gpu_l2(w, parity=P == 6))
        assert r[1] < r[0], (P, r)


def test_p_convergence_variable_velocity_explicit_step():
    """Section 5.2, Fig. fig:2_2a (H = 4, T = 1, explicit step, P = 3..12)."""
    Ps = list(range(3, 13))
    err = {c: np.array([_gpu_l2(W.x6(P=P, H=4, rk=rk, cmask=cm), parity=P in (5, 12)) for P in Ps])
           for c, (rk, cm) in CASES.items()}
    # first order: algebraic (less than 20x from P = 3 to 12)
    for c in ("Basecase1", "MF1"):
        assert err[c][0] / err[c][-1] < 20 and np.all(err[c][1:] < err[c][:-1])
    # second order: more than 500x from P = 3 to 10, then bound by the time error
    for c in ("Basecase2", "MF2"):
        assert err[c][0] / err[c][Ps.index(10)] > 500
        assert err[c][Ps.index(10)] / err[c][-1] < 5
    # third order: converges furthest, below 5e-6 at P = 12
    assert err["MF3"][-1] < 5e-6 and err["MF3"][-1] < err["MF2"][-1] / 5


def test_p_convergence_variable_velocity_small_step():
    """Section 5.2, Fig. fig:2_2b (dt = 1e-4, T = 1): the first-order scheme
    converges spectrally up to P = 8, where its error is O(1e-4), and is then
    bound by the time integration; the second-order one keeps converging."""
    Ps = list(range(4, 12))
    e1, e2 = [], []
    for P in Ps:
        for rk, out in ((1, e1), (2, e2)):
            w = W.x6(P=P, H=4, rk=rk, cmask=W.BOUNDARY)
            w.dt, w.nsteps = 1e-4, 10000
            out.append(_gpu_l2(w, parity=P == 8))
    e1, e2 = np.array(e1), np.array(e2)
    i8 = Ps.index(8)
    assert e1[0] / e1[i8] > 30                       # spectral to P = 8
    assert 1e-4 < e1[i8] < 1e-3                       # O(1e-4) there
    assert e1[i8] / e1[-1] < 1.5                      # then bound
    assert e2[-1] < e1[-1] / 10 and e2[-1] < 2e-5     # second order keeps going
