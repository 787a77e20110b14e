"""GPU tests of the request loop (sl_server_*): each result is the same
alone and in the mix (bit for bit: every kernel is deterministic and works
per mesh), batched and one stream per request alike, batches that carry
several requests' steps per launch, admission by slots and memory budget,
failure isolation, latency statistics, and one request against the oracle."""
import math

import numpy as np
import pytest

import workloads as W
from _parity import announce, rel_l2, run_oracle

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _need_gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1910_06476_amd as P
    P.lib()


def _requests(seed=0, count=8):
    """A seeded mix of 1D and 2D problems of different sizes, orders,
    boundary types, forms, constraint sets and precisions."""
    rng = np.random.default_rng(seed)
    reqs = []
    for i in range(count):
        dim = 1 if i % 2 == 0 else 2
        if dim == 1:
            K = int(rng.integers(16, 600))
            n = int(rng.integers(5, 18))
            w = W.c2(K=K, n=n, nsteps=int(rng.integers(3, 12)),
                     cmask=[W.BOUNDARY, W.BOUNDARY | W.MASS, W.BOUNDARY | W.MASS | W.ENERGY][i % 3])
            w.energy_maxit, w.energy_tol = 3, 0.0
            prec = 0
        else:
            k = int(rng.integers(3, 14))
            n = int(rng.integers(4, 11))
            w = W.c3(kx=k, ky=k, n=n, nsteps=int(rng.integers(3, 10)))
            prec = int(i % 4 == 1)  # some in FP32-refined
        reqs.append((w, prec))
    return reqs


def _submit(S, w, prec, dt=None):
    import paper_1910_06476_amd as P
    a, _ = w.velocity()
    ghost = w.ghost_rows(0.0, w.nsteps) if w.bc == W.GHOST else None
    return S.submit(w.dim, w.kx, w.ky, w.n - 1, w.initial(), a, dt=w.dt if dt is None else dt, nsteps=w.nsteps,
                    ghost=ghost, nodes=w.family, bc=w.bc, form=w.form, precision=prec, x0=w.x0, x1=w.x1,
                    y0=w.y0, y1=w.y1, rk=w.rk, constraints=w.cmask, mode=w.mode, energy_maxit=w.energy_maxit,
                    energy_tol=w.energy_tol)


def _alone(w, prec):
    import paper_1910_06476_amd as P
    with P.Server(max_active=1) as S:
        rid = _submit(S, w, prec)
        S.drain()
        return S.result(rid)


@pytest.mark.parametrize("max_active", [2, 4, 8])
def test_alone_and_in_the_mix_are_identical(max_active):
    import paper_1910_06476_amd as P
    reqs = _requests(seed=max_active)
    alone = [_alone(w, p) for w, p in reqs]
    announce(f"serve mix max_active={max_active}")
    with P.Server(max_active=max_active) as S:
        ids = [_submit(S, w, p) for w, p in reqs]
        S.drain()
        mixed = [S.result(i) for i in ids]
    for (rc0, f0, st0, _), (rc1, f1, st1, _) in zip(alone, mixed):
        assert rc0 == rc1
        assert np.array_equal(f0, f1)
        assert st0.flags == st1.flags and st0.max_picard == st1.max_picard


def _run(reqs, max_active, batch):
    import paper_1910_06476_amd as P
    with P.Server(max_active=max_active, batch=batch) as S:
        ids = [_submit(S, w, p) for w, p in reqs]
        S.drain()
        out = [S.result(i) for i in ids]
        return out, S.batching()


@pytest.mark.parametrize("seed", [11, 12])
def test_batched_and_unbatched_are_identical(seed):
    """The same mix through batched launches and through one stream per
    request: the same fields, bit for bit, and the same statistics."""
    reqs = _requests(seed=seed, count=10)
    announce(f"serve batched vs unbatched seed={seed}")
    a, (launches_a, steps_a) = _run(reqs, 6, True)
    b, (launches_b, steps_b) = _run(reqs, 6, False)
    assert launches_b == 0 and steps_b == 0
    assert steps_a > 0
    for (rc0, f0, st0, _), (rc1, f1, st1, _) in zip(a, b):
        assert rc0 == rc1 == 0
        assert np.array_equal(f0, f1)
        assert st0.flags == st1.flags and st0.max_picard == st1.max_picard
        assert st0.steps == st1.steps


@pytest.mark.parametrize("dim", [1, 2])
def test_requests_of_one_variant_share_launches(dim):
    """Requests of one kernel variant admitted together are stepped by
    shared launches: one group step per step of the longest request, each
    carrying every request that still has steps left; each result equals
    the request stepped alone."""
    import paper_1910_06476_amd as P
    rng = np.random.default_rng(dim)
    reqs = []
    for i in range(5):
        steps = int(rng.integers(3, 9))
        if dim == 1:
            w = W.c2(K=int(rng.integers(20, 400)), n=13, nsteps=steps, cmask=W.BOUNDARY)
        else:
            k = int(rng.integers(3, 10))
            w = W.c3(kx=k, ky=k, n=9, nsteps=steps)
        reqs.append((w, 0))
    announce(f"serve one variant dim={dim}")
    out, (launches, member_steps) = _run(reqs, 8, True)
    assert member_steps == sum(w.nsteps for w, _ in reqs)
    assert launches == max(w.nsteps for w, _ in reqs)
    for (w, p), (rc, f, st, _) in zip(reqs, out):
        rc0, f0, st0, _ = _alone(w, p)
        assert rc == rc0 == 0
        assert np.array_equal(f, f0)


def test_memory_budget_admits_in_order():
    """A budget that holds only the largest request at a time: requests run
    one after another, in arrival order, with the same results."""
    import paper_1910_06476_amd as P
    reqs = _requests(seed=11, count=5)
    sizes = [P.sl_mesh_bytes(w.dim, w.kx, w.ky, w.n - 1, bc=w.bc, ghost_rows=w.nsteps + 1 if w.bc == W.GHOST else 0)
             for w, _ in reqs]
    budget = max(sizes)
    announce("serve budget")
    with P.Server(max_active=8, hbm_budget=budget) as S:
        ids = [_submit(S, w, p) for w, p in reqs]
        seen_active = []
        while True:
            a, q = S.progress()
            seen_active.append(a)
            if a == 0 and q == 0:
                break
        res = [S.result(i) for i in ids]
    assert max(seen_active) >= 1
    for (w, p), (rc, f, st, tm) in zip(reqs, res):
        rc0, f0, _, _ = _alone(w, p)
        assert rc == rc0 and np.array_equal(f, f0)
        assert tm.bytes <= budget
    # admitted in arrival order, one at a time
    assert [r[3].admit_seq for r in res] == list(range(len(res)))


def test_failed_request_is_isolated():
    """A request whose dt breaks the time-step restriction fails with
    SL_E_CFL; the others complete as if alone."""
    import paper_1910_06476_amd as P
    reqs = _requests(seed=3, count=4)
    announce("serve failure isolation")
    with P.Server(max_active=4) as S:
        ids = []
        for k, (w, p) in enumerate(reqs):
            ids.append(_submit(S, w, p, dt=w.dt * 1e3 if k == 1 else None))
        S.drain()
        res = [S.result(i) for i in ids]
    assert res[1][0] == P.SL_E_CFL
    for k in (0, 2, 3):
        rc0, f0, _, _ = _alone(*reqs[k])
        assert res[k][0] == rc0 and np.array_equal(res[k][1], f0)


def test_latency_statistics():
    import paper_1910_06476_amd as P
    reqs = _requests(seed=5, count=6)
    announce("serve latency")
    with P.Server(max_active=3) as S:
        ids = [_submit(S, w, p) for w, p in reqs]
        S.drain()
        p50, p99, n, dof = S.latency()
        for i in ids:
            S.result(i)
    assert n == sum(w.nsteps for w, _ in reqs)
    assert 0.0 < p50 <= p99
    assert dof == sum(w.K * w.nd * w.nsteps for w, _ in reqs)


def test_served_request_matches_oracle():
    import paper_1910_06476_amd as P
    w = W.c3(kx=6, ky=6, n=7, nsteps=4)
    announce("serve vs oracle")
    rc, g, st, tm = _alone(w, 0)
    o, ost = run_oracle(w)
    assert rc == 0
    assert rel_l2(g, o) <= 1e-12
