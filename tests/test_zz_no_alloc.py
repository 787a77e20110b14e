"""The allocation-free 1D entry point (sl_step1d_static: caller device
buffers, scratch in the library's fixed device array) against the existing
entry point (sl_create_mesh + sl_set_velocity + sl_step + sl_read) on the
same data, through the C-ABI: two calls in a row, the second smaller, then
the first again (the shared scratch keeps no state that changes a result)."""
import numpy as np
import pytest

import workloads as W
from _parity import announce, assert_parity, opts_dict, run_gpu
from test_gpu_1d import _case

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _need_gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1910_06476_amd as P
    P.lib()


def _run_static(w, nsteps):
    import torch
    import paper_1910_06476_amd as P
    dev = torch.device("cuda:0")
    phi = torch.tensor(w.initial(), dtype=torch.float64, device=dev)
    out = torch.full_like(phi, float("nan"))
    a_np, _ = w.velocity()
    a = torch.tensor(a_np, dtype=torch.float64, device=dev)
    ghost = None
    if w.bc != W.PERIODIC:
        ghost = torch.tensor(np.asarray(w.ghost_rows(0.0, nsteps), dtype=np.float64).ravel()[:2 * (nsteps + 1)],
                             device=dev)
    stats = torch.full((4,), -1.0, dtype=torch.float64, device=dev)
    flags = torch.full((1,), -1, dtype=torch.int32, device=dev)
    o = P.step_opts(**opts_dict(w))
    P.sl_step1d_static(w.K, w.n - 1, phi.data_ptr(), out.data_ptr(), a.data_ptr(), float(np.abs(a_np).max()),
                       w.dt, nsteps, opts=o, ghost=ghost.data_ptr() if ghost is not None else 0,
                       nodes=w.family, bc=w.bc, form=w.form, x0=w.x0, x1=w.x1, stats=stats.data_ptr(),
                       flags=flags.data_ptr(), stream=torch.cuda.current_stream().cuda_stream)
    torch.cuda.synchronize()
    return out.cpu().numpy(), stats.cpu().numpy(), int(flags.cpu().item())


def _check(w, nsteps):
    g, st, flags = _run_static(w, nsteps)
    ref, rst, rc = run_gpu(w, nsteps=nsteps)
    assert_parity(w, g, ref)
    assert flags == rst.flags
    assert int(st[3]) == rst.max_picard
    np.testing.assert_allclose(st[:3], [rst.resid_boundary, rst.resid_mass, rst.resid_energy], rtol=0,
                               atol=1e-12 * max(1.0, float(np.abs(ref).max())))
    return g


def test_static_matches_mesh_path_two_calls():
    w1 = W.c2(K=4096, nsteps=3)  # C2 shape: boundary + mass + energy HARD, tol 1e-8
    announce("static 1D K=4096 n=17 B+M+E 3 steps")
    first = _check(w1, 3)
    w2 = _case(n=9, K=300, bc=W.GHOST, cmask=W.BOUNDARY | W.MASS | W.ENERGY, mode=W.SOFT)
    announce("static 1D K=300 n=9 ghost SOFT 3 steps")
    _check(w2, 3)
    announce("static 1D K=4096 n=17 again")
    again, _, _ = _run_static(w1, 3)
    np.testing.assert_array_equal(again, first)


def test_static_even_step_count_and_in_place():
    """An even step count ends in phi_out through the scratch field, and
    phi_out may be phi_in."""
    import torch
    import paper_1910_06476_amd as P
    w = _case(n=17, K=37, cmask=W.BOUNDARY | W.MASS)
    announce("static 1D K=37 n=17 2 steps in place")
    ref, rst, rc = run_gpu(w, nsteps=2)
    dev = torch.device("cuda:0")
    phi = torch.tensor(w.initial(), dtype=torch.float64, device=dev)
    a_np, _ = w.velocity()
    a = torch.tensor(a_np, dtype=torch.float64, device=dev)
    P.sl_step1d_static(w.K, w.n - 1, phi.data_ptr(), phi.data_ptr(), a.data_ptr(), float(np.abs(a_np).max()),
                       w.dt, 2, opts=P.step_opts(**opts_dict(w)), x0=w.x0, x1=w.x1,
                       stream=torch.cuda.current_stream().cuda_stream)
    torch.cuda.synchronize()
    assert_parity(w, phi.cpu().numpy(), ref)
