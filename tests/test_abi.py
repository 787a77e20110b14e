"""C-ABI checks that need no GPU: the library loads, exports every entry
point include/sl.h declares, and its host-only functions behave (node tables
against numpy's library rules, status strings, descriptor validation that
fails before any device call)."""
import ctypes
import os
import re

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def sl():
    import paper_1910_06476_amd as P
    if not os.path.exists(P.LIBPATH):
        pytest.skip("libsl.so not built (run __graft_entry__.build())")
    return P


def declared_functions():
    src = open(os.path.join(ROOT, "include", "sl.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(sl_[a-z_0-9]+)\s*\(", src)))


def test_exports_every_declared_symbol(sl):
    names = declared_functions()
    assert len(names) >= 12
    L = ctypes.CDLL(sl.LIBPATH)
    for name in names:
        assert hasattr(L, name), name
    assert sorted(sl.EXPORTS) == names


@pytest.mark.parametrize("n", range(1, 33))
def test_node_coords_gauss_legendre(sl, n):
    xi, w = sl.sl_node_coords(sl.SL_NODES_GL, n)
    t, wl = np.polynomial.legendre.leggauss(n)
    order = np.argsort((1 - t) / 2)
    np.testing.assert_allclose(xi, ((1 - t) / 2)[order], atol=3e-16)
    np.testing.assert_allclose(w, (wl / 2)[order], atol=3e-15)


@pytest.mark.parametrize("n", range(1, 20))
def test_node_coords_chebyshev_gauss(sl, n):
    xi, w = sl.sl_node_coords(sl.SL_NODES_CG, n)
    t, _ = np.polynomial.chebyshev.chebgauss(n)
    np.testing.assert_allclose(xi, np.sort((1 - t) / 2), atol=3e-16)
    for k in range(n):  # interpolatory: exact below degree n
        assert abs(np.dot(w, xi ** k) - 1 / (k + 1)) < 1e-13


def test_node_coords_rejects(sl):
    with pytest.raises(sl.SLError):
        sl.sl_node_coords(7, 5)
    with pytest.raises(sl.SLError):
        sl.sl_node_coords(0, 0)


def test_status_strings(sl):
    for s in range(9):
        assert isinstance(sl.status_string(s), str) and sl.status_string(s)
    assert sl.status_string(99) == "unknown status"


@pytest.mark.parametrize("bad", [
    dict(dim=3), dict(order=0), dict(order=17), dict(kx=0), dict(ky=2), dict(nodes=5), dict(bc=2), dict(bc=3),
    dict(bc=4),
    dict(form=2), dict(precision=1), dict(precision=2), dict(precision=3), dict(x1=0.0),
])
def test_create_mesh_validates_before_touching_the_device(sl, bad):
    args = dict(dim=1, kx=4, ky=1, order=3, nodes=0, bc=0, form=0, precision=0, x0=0.0, x1=1.0)
    args.update(bad)
    u0 = np.zeros(4 * 4 * 4)
    with pytest.raises(sl.SLError) as ei:
        sl.sl_create_mesh(args.pop("dim"), args.pop("kx"), args.pop("ky"), args.pop("order"), u0, **args)
    assert ei.value.status == sl.SL_E_INVALID


def test_null_handles_rejected(sl):
    L = sl.lib()
    assert L.sl_step(None, 0.1, 1, None) == sl.SL_E_INVALID
    assert L.sl_read(None, None, None) == sl.SL_E_INVALID
    assert L.sl_destroy_mesh(None) == sl.SL_E_INVALID
    assert L.sl_set_velocity(None, None, None) == sl.SL_E_INVALID
    assert L.sl_max_dt(None, 1.0) == 0.0
    assert L.sl_ghost_count(None) == 0


def test_mesh_bytes_host_only(sl):
    b1 = sl.sl_mesh_bytes(1, 1000, 1, 8)
    b2 = sl.sl_mesh_bytes(1, 2000, 1, 8)
    assert 0 < b1 < b2 <= 2 * b1 + 4096
    # 1D: three fields, two velocity arrays, two divergence arrays at least
    assert b1 >= 7 * 1000 * 9 * 8
    g0 = sl.sl_mesh_bytes(2, 16, 16, 4, bc=sl.SL_BC_GHOST, ghost_rows=0)
    g3 = sl.sl_mesh_bytes(2, 16, 16, 4, bc=sl.SL_BC_GHOST, ghost_rows=3)
    assert g3 - g0 == 3 * 2 * 5 * (16 + 16) * 8
    with pytest.raises(sl.SLError):
        sl.sl_mesh_bytes(2, 4, 4, 17)  # 18 nodes per direction: beyond the 2D limit
    with pytest.raises(sl.SLError):
        sl.sl_mesh_bytes(1, 4, 2, 4)   # 1D with ky != 1


def test_server_host_side_validation(sl):
    """Creation, submission and result lookup are host-only: descriptor
    checks, the budget check and the request table."""
    with pytest.raises(sl.SLError):
        sl.Server(max_active=0)
    with pytest.raises(sl.SLError):
        sl.Server(max_active=65)
    h = ctypes.c_void_p()
    assert sl.lib().sl_server_create(ctypes.byref(sl.ServerDesc(2, 2, 1 << 20)), ctypes.byref(h)) == sl.SL_E_INVALID
    sl.Server(max_active=2, batch=False).close()
    s = sl.Server(max_active=2, hbm_budget=1 << 20)
    try:
        n = 5
        u0 = np.zeros(4096 * n)
        a = np.ones(4096 * n)
        with pytest.raises(sl.SLError) as e:  # needs more than the 1 MiB budget
            s.submit(1, 4096, 1, n - 1, u0, a, dt=1e-4, nsteps=1)
        assert e.value.status == sl.SL_E_NOMEM
        rid = s.submit(1, 16, 1, n - 1, np.zeros(16 * n), np.ones(16 * n), dt=1e-4, nsteps=1)
        with pytest.raises(sl.SLError) as e:  # waiting, not finished
            s.result(rid)
        assert e.value.status == sl.SL_E_STATE
        with pytest.raises(sl.SLError):
            s.result(rid + 100)
        with pytest.raises(sl.SLError):  # ghost mesh without ghost rows
            s.submit(1, 16, 1, n - 1, np.zeros(16 * n), np.ones(16 * n), dt=1e-4, nsteps=1, bc=sl.SL_BC_GHOST)
        # a mixed-order descriptor (mesh.orders set) is refused: requests are
        # sized as uniform meshes
        kx = ky = 2
        orders = np.array([3, 4, 3, 4], dtype=np.int32)
        dofs = int(((orders + 1) ** 2).sum())
        u0, av = np.zeros(dofs), np.ones(2 * dofs)
        q = sl.Request()
        q.mesh = sl.MeshDesc(dim=2, kx=kx, ky=ky, order=3, nodes=0, bc=0, form=0, precision=0, x0=0.0, x1=1.0,
                             y0=0.0, y1=1.0, u0=u0.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), stream=None,
                             orders=orders.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)))
        q.a = av.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
        q.nsteps, q.dt, q.opts = 1, 1e-4, sl.step_opts()
        rid = ctypes.c_int64(-1)
        assert sl.lib().sl_server_submit(s.h, ctypes.byref(q), ctypes.byref(rid)) == sl.SL_E_INVALID
    finally:
        s.close()


def test_step1d_static_rejects_before_any_device_call(sl):
    """The allocation-free 1D entry point refuses sizes beyond its scratch
    array (65536 elements, order 16) and bad arguments with SL_E_INVALID,
    before touching the device (this runs without a GPU)."""
    L = sl.lib()
    one = ctypes.c_void_p(16)  # never dereferenced: validation fails first
    o = sl.step_opts()
    cases = [
        dict(K=65537, order=16), dict(K=0, order=4), dict(K=100, order=17), dict(K=100, order=0),
        dict(K=100, order=4, nsteps=-1), dict(K=100, order=4, dt=0.0), dict(K=100, order=4, bc=2),
        dict(K=100, order=4, nodes=3), dict(K=100, order=4, x1=0.0), dict(K=100, order=4, amax=-1.0),
    ]
    for c in cases:
        K, order = c["K"], c["order"]
        rc = L.sl_step1d_static(K, order, c.get("nodes", 0), c.get("bc", 0), 0, 0.0, c.get("x1", 1.0), one, one,
                                one, None, c.get("amax", 1.0), None, c.get("dt", 1e-6), c.get("nsteps", 1),
                                ctypes.byref(o), None, None, None)
        assert rc == sl.SL_E_INVALID, c
    # a NULL field pointer, and a ghost mesh without ghost rows
    assert L.sl_step1d_static(100, 4, 0, 0, 0, 0.0, 1.0, None, one, one, None, 1.0, None, 1e-6, 1,
                              ctypes.byref(o), None, None, None) == sl.SL_E_INVALID
    assert L.sl_step1d_static(100, 4, 0, 1, 0, 0.0, 1.0, one, one, one, None, 1.0, None, 1e-6, 1,
                              ctypes.byref(o), None, None, None) == sl.SL_E_INVALID
    # the time-step restriction, as sl_step
    assert L.sl_step1d_static(100, 4, 0, 0, 0, 0.0, 1.0, one, one, one, None, 1.0, None, 1e-2, 1,
                              ctypes.byref(o), None, None, None) == sl.SL_E_CFL
