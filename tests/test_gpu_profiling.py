"""Per-kernel timing through the C-ABI (sl_set_profiling, sl_kernel_time).

Timed launches record the start and end of their own dispatch.  Profiled
steps must give the same field, bit for bit, as unprofiled ones; every
launch of a timed kernel is counted once, with a positive duration, and the
durations of the kernels of a step fit inside the steps' wall time."""
import time

import numpy as np
import pytest

import workloads as W
from _parity import announce, opts_dict

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _need_gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1910_06476_amd as P
    P.lib()


def _run(w, nsteps, kinds, profiling, mixed=False, ghost=False, **over):
    import torch
    import paper_1910_06476_amd as P
    m = P.from_mixed_workload(w) if mixed else P.from_workload(w)
    try:
        if ghost:
            m.set_ghost(w.ghost_rows(0.0, nsteps))
        opts = dict(rk=w.rk, constraints=W.BOUNDARY, mode=w.mode) if mixed else opts_dict(w, **over)
        if profiling:
            P.sl_set_profiling(m.h, True)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        m.step(w.dt, nsteps, **opts)
        rc, out, st = m.read()
        wall_ms = (time.perf_counter() - t0) * 1e3
        times = {k: P.sl_kernel_time(m.h, k) for k in kinds} if profiling else {}
    finally:
        m.close()
    return np.asarray(out), rc, times, wall_ms


def _check(w, nsteps, kinds, mixed=False, ghost=False, **over):
    a, rc_a, _, _ = _run(w, nsteps, kinds, False, mixed, ghost, **over)
    b, rc_b, times, wall = _run(w, nsteps, kinds, True, mixed, ghost, **over)
    assert rc_a == rc_b == 0
    assert np.array_equal(a, b)
    total = 0.0
    for k, (ms, count) in times.items():
        assert count == nsteps, (k, count)
        assert np.isfinite(ms) and ms > 0, (k, ms)
        total += ms
    assert total < wall, (total, wall)


def test_profiled_1d_steps():
    import paper_1910_06476_amd as P
    w = W.c2(K=512, nsteps=6)
    announce("profiling 1D K=512 n=17 B+M+E 6 steps")
    _check(w, 6, [P.KER_ADV1D, P.KER_CON1D])


def test_profiled_2d_steps():
    import paper_1910_06476_amd as P
    w = W.c3(kx=16, nsteps=5)
    announce("profiling 2D 16x16 n=9 ghost inflow 5 steps")
    _check(w, 5, [P.KER_ADV2D, P.KER_CON2D], ghost=True)


def test_profiled_2d_targets_and_backtraces():
    import paper_1910_06476_amd as P
    w = W.c3(kx=16, nsteps=5)
    w.cmask = W.BOUNDARY | W.MASS | W.ENERGY
    announce("profiling 2D 16x16 n=9 B+M+E backtracked faces 5 steps")
    _check(w, 5, [P.KER_ADV2D, P.KER_CON2D, P.KER_TGT2D, P.KER_BT2D], ghost=True, iface=P.SL_IFACE_BACKTRACK)


def test_profiled_mixed_steps():
    import paper_1910_06476_amd as P
    w = W.c4(kx=12, nsteps=4)
    nb = len(set(w.orders.tolist()))
    announce(f"profiling mixed 12x12 {nb} buckets 4 steps")
    kinds = [P.KER_MIX_ADV + b for b in range(nb)] + [P.KER_MIX_CON + b for b in range(nb)]
    _check(w, 4, kinds, mixed=True)
