"""Paper parity of the oracle: the numbers printed in Tables 2 and 3.

Readings that reproduce them (all in the design notes): n = P + 1
Chebyshev-Gauss nodes per element; dt = (edge-to-first-node gap) * dx /
|u|max; floor(T/dt) full steps; the literal stacked least squares of eq.
matrix_a (SOFT); the paper's L2 norm with physical dx (eq. 5.2); ||M||, ||E||
as ratios of global integrals; second order = Heun, third order = Kutta.
The oracle runs with nodal (interpolated) velocity here, exactly the model
the HIP path uses.
"""
import math
import os

import numpy as np
import pytest

import workloads as W

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def _rows(name):
    out = []
    for line in open(os.path.join(GOLD, name)):
        line = line.strip()
        if line and not line.startswith("#"):
            out.append(line.split())
    return out


def _sig(x, like):
    """round x to the number of significant digits of the printed string"""
    mant = like.lower().split("e")[0].lstrip("-")
    digits = len(mant.replace(".", "").lstrip("0")) or 1
    if "e" in like.lower():
        return float("%.*e" % (digits - 1, x))
    dec = len(mant.split(".")[1]) if "." in mant else 0
    return round(x, dec)


def _paper_norms(ora, w, phi, t):
    xi, wq = ora.nodes(w.family, w.n)
    x = w.x0 + (np.arange(w.K)[:, None] + xi[None, :]) * w.dx
    ex = w.exact(x, None, t)
    P = phi.reshape(w.K, w.n)
    l2 = np.sqrt(((P - ex) ** 2 * wq * w.dx).sum(1)).sum()
    M = (P * wq).sum() / (ex * wq).sum()
    E = (P ** 2 * wq).sum() / (ex ** 2 * wq).sum()
    return l2, M - 1.0, E


def test_table2_basecase_h_convergence(ora):
    """R-PIN-1: Table 2 (tab:h_conv), Basecase, P=4, H=5,6,7, T=10."""
    rows = _rows("table2_basecase.txt")
    errs = {}
    for H in (4, 5, 6, 7):
        w = W.x1(P=4, H=H, rk=1)
        phi, st = ora.run_workload(w)
        assert st.flags == 0
        errs[H] = _paper_norms(ora, w, phi, w.nsteps * w.dt)[0]
    for H, l2, slope in rows:
        H = int(H)
        assert _sig(errs[H], l2) == float(l2), (H, errs[H], l2)
        s = math.log(errs[H - 1] / errs[H]) / math.log(H / (H - 1))
        assert abs(s - float(slope)) <= 0.02, (H, s, slope)


@pytest.mark.parametrize("case", ["Basecase1", "Basecase2", "MF2", "MF3"])
def test_table3_pinned_rows(ora, case):
    """R-PIN-2: Table 3 (tab:3), phi_t + (-sin(x) phi)_x = 0, H=4, P=6, T=1."""
    spec = {"Basecase1": (1, W.BOUNDARY), "Basecase2": (2, W.BOUNDARY),
            "MF2": (2, W.BOUNDARY | W.MASS), "MF3": (3, W.BOUNDARY | W.MASS)}[case]
    row = [r for r in _rows("table3.txt") if r[0] == case][0]
    assert row[4] == "pinned"
    w = W.x6(rk=spec[0], cmask=spec[1])
    phi, st = ora.run_workload(w)
    assert st.flags & ~ora.F_CONTAIN == 0
    l2, dm, e = _paper_norms(ora, w, phi, w.nsteps * w.dt)
    assert _sig(dm, row[1]) == float(row[1]) or (float(row[1]) == 0 and abs(dm) < 5e-5)
    assert _sig(e, row[2]) == float(row[2])
    assert _sig(l2, row[3]) == float(row[3]), (case, l2)


def test_table3_first_order_mass_row_is_not_reproduced(ora):
    """MF1 / MEF rows are parity-unpinned: record that the oracle's MF1
    differs from the printed row, so a later change that happens to match it
    is noticed and examined."""
    row = [r for r in _rows("table3.txt") if r[0] == "MF1"][0]
    w = W.x6(rk=1, cmask=W.BOUNDARY | W.MASS)
    phi, _ = ora.run_workload(w)
    l2, dm, e = _paper_norms(ora, w, phi, w.nsteps * w.dt)
    assert _sig(l2, row[3]) != float(row[3])


def test_basecase_independent_of_integrator_for_constant_velocity(ora):
    """Section 5.1: with constant velocity the particle positions are exact for
    any RK order, so Basecase results do not depend on the integrator."""
    outs = []
    for rk in (1, 2, 3, 4):
        w = W.x1(P=5, H=4, rk=rk, T=0.5)
        phi, _ = ora.run_workload(w)
        outs.append(phi)
    for o in outs[1:]:
        np.testing.assert_allclose(o, outs[0], atol=1e-13)


def _l2(ora, w, phi):
    return _paper_norms(ora, w, phi, w.nsteps * w.dt)[0]


def test_dirichlet_more_accurate_than_periodic(ora):
    """Section 5.1 (Fig. fig:1_3): Basecase with exact inflow (Dirichlet)
    values against periodic, H = 4, T = 10: the Dirichlet error is lower at
    every P (here by about 10x; the paper's figure shows it slightly lower)."""
    for P in (4, 6, 8):
        r = []
        for bc in (W.PERIODIC, W.GHOST):
            w = W.x1(P=P, H=4, rk=1)
            w.bc = bc
            phi, st = ora.run_workload(w)
            assert st.flags == 0
            r.append(_l2(ora, w, phi))
        assert r[1] < r[0], (P, r)


def test_first_order_bounded_by_time_error_at_small_step(ora):
    """Section 5.2 (Fig. fig:2_2b): with dt = 1e-4 the first-order Basecase
    converges spectrally up to P = 8, where its error is O(1e-4), and is then
    bound by the time integration; the second-order Basecase keeps
    converging."""
    e1, e2 = {}, {}
    for P in (4, 8, 11):
        for rk, out in ((1, e1), (2, e2)):
            w = W.x6(P=P, H=4, rk=rk, cmask=W.BOUNDARY)
            w.dt, w.nsteps = 1e-4, 10000
            phi, _ = ora.run_workload(w)
            out[P] = _l2(ora, w, phi)
    assert e1[4] / e1[8] > 30 and 1e-4 < e1[8] < 1e-3 and e1[8] / e1[11] < 1.5
    assert e2[11] < e1[11] / 10
