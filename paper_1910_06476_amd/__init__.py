"""Python binding of the MI355X semi-Lagrangian spectral transport library.

Argument marshalling only: every step of the method runs in the HIP kernels
of ``libsl.so`` (built in-tree by ``build.py``), called through the C ABI
declared in ``include/sl.h``.  The function names mirror the C entry points;
``Mesh`` is a small convenience wrapper that owns one ``sl_mesh``.

Importing this package does not need a GPU, but it needs the built library:
if ``libsl.so`` is missing the import fails with an explicit error -- there
is no fallback implementation.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIBPATH = os.path.join(_HERE, "libsl.so")

SL_OK, SL_E_INVALID, SL_E_NOMEM, SL_E_DEVICE, SL_E_STATE, SL_E_CFL, SL_E_NONFINITE, SL_E_SINGULAR, SL_E_NOCONV = range(9)
SL_NODES_GL, SL_NODES_CG = 0, 1
SL_BC_PERIODIC, SL_BC_GHOST, SL_BC_PERIODIC_X, SL_BC_PERIODIC_Y = 0, 1, 2, 3
SL_FORM_ADVECTIVE, SL_FORM_CONSERVATIVE = 0, 1
SL_PREC_FP64, SL_PREC_FP32_REFINED, SL_PREC_BF16_REFINED = 0, 1, 2
SL_C_BOUNDARY, SL_C_MASS, SL_C_ENERGY = 1, 2, 4
SL_MODE_HARD, SL_MODE_SOFT = 0, 1
SL_IFACE_INTERP, SL_IFACE_BACKTRACK = 0, 1
SL_SERVER_NO_BATCH = 1
KER_ADV1D, KER_CON1D, KER_ADV2D, KER_CON2D = 0, 1, 2, 3
KER_MIX_ADV, KER_MIX_CON = 4, 20  # + bucket index (mixed-order meshes)
KER_TGT2D, KER_BT2D = 36, 37  # uniform 2D: mass/energy targets, face backtraces

EXPORTS = ["sl_create_mesh", "sl_set_velocity", "sl_set_ghost", "sl_ghost_count", "sl_step", "sl_read",
           "sl_destroy_mesh", "sl_status_string", "sl_max_dt", "sl_node_coords", "sl_device_field",
           "sl_set_profiling", "sl_kernel_time", "sl_mesh_bytes", "sl_server_create", "sl_server_submit",
           "sl_server_progress", "sl_server_drain", "sl_server_result", "sl_server_latency",
           "sl_server_destroy", "sl_step1d_static", "sl_bucket_stats", "sl_server_batching"]


class MeshDesc(ctypes.Structure):
    _fields_ = [("dim", ctypes.c_int32), ("kx", ctypes.c_int32), ("ky", ctypes.c_int32),
                ("order", ctypes.c_int32), ("nodes", ctypes.c_int32), ("bc", ctypes.c_int32),
                ("form", ctypes.c_int32), ("precision", ctypes.c_int32),
                ("x0", ctypes.c_double), ("x1", ctypes.c_double), ("y0", ctypes.c_double),
                ("y1", ctypes.c_double), ("u0", ctypes.POINTER(ctypes.c_double)), ("stream", ctypes.c_void_p),
                ("orders", ctypes.POINTER(ctypes.c_int32))]


class StepOpts(ctypes.Structure):
    _fields_ = [("rk", ctypes.c_int32), ("constraints", ctypes.c_int32), ("mode", ctypes.c_int32),
                ("energy_maxit", ctypes.c_int32), ("refine_steps", ctypes.c_int32),
                ("iface", ctypes.c_int32), ("energy_tol", ctypes.c_double)]


class Stats(ctypes.Structure):
    _fields_ = [("t", ctypes.c_double), ("steps", ctypes.c_int64), ("mass", ctypes.c_double),
                ("energy", ctypes.c_double), ("resid_boundary", ctypes.c_double),
                ("resid_mass", ctypes.c_double), ("resid_energy", ctypes.c_double),
                ("refine_resid", ctypes.c_double), ("max_picard", ctypes.c_int32), ("flags", ctypes.c_int32),
                ("vel_terms", ctypes.c_int32), ("remap_sweeps_max", ctypes.c_int32),
                ("remap_sweeps_mean", ctypes.c_double)]

    def asdict(self):
        return {f: getattr(self, f) for f, _ in self._fields_}


class ServerDesc(ctypes.Structure):
    _fields_ = [("max_active", ctypes.c_int32), ("flags", ctypes.c_int32), ("hbm_budget", ctypes.c_size_t)]


class Request(ctypes.Structure):
    _fields_ = [("mesh", MeshDesc), ("a", ctypes.POINTER(ctypes.c_double)),
                ("div_a", ctypes.POINTER(ctypes.c_double)), ("ghost", ctypes.POINTER(ctypes.c_double)),
                ("ghost_rows", ctypes.c_int32), ("nsteps", ctypes.c_int32), ("dt", ctypes.c_double),
                ("opts", StepOpts)]


class RequestTiming(ctypes.Structure):
    _fields_ = [("queue_us", ctypes.c_double), ("total_us", ctypes.c_double), ("device_ms", ctypes.c_double),
                ("bytes", ctypes.c_size_t), ("admit_seq", ctypes.c_int64)]


class SLError(RuntimeError):
    def __init__(self, status: int, where: str):
        self.status = status
        super().__init__(f"{where}: {status_string(status)} ({status})")


_lib = None


def lib():
    """Load libsl.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIBPATH):
            raise ImportError(f"{LIBPATH} is missing: build it with "
                              "`python paper_1910_06476_amd/build.py` (no fallback exists)")
        L = ctypes.CDLL(LIBPATH)
        dp = ctypes.POINTER(ctypes.c_double)
        vp = ctypes.c_void_p
        L.sl_create_mesh.argtypes = [ctypes.POINTER(MeshDesc), ctypes.POINTER(vp)]
        L.sl_set_velocity.argtypes = [vp, dp, dp]
        L.sl_set_ghost.argtypes = [vp, dp, ctypes.c_int32]
        L.sl_ghost_count.argtypes = [vp]
        L.sl_ghost_count.restype = ctypes.c_int32
        L.sl_step.argtypes = [vp, ctypes.c_double, ctypes.c_int32, ctypes.POINTER(StepOpts)]
        L.sl_read.argtypes = [vp, dp, ctypes.POINTER(Stats)]
        L.sl_destroy_mesh.argtypes = [vp]
        L.sl_status_string.argtypes = [ctypes.c_int32]
        L.sl_status_string.restype = ctypes.c_char_p
        L.sl_max_dt.argtypes = [vp, ctypes.c_double]
        L.sl_max_dt.restype = ctypes.c_double
        L.sl_node_coords.argtypes = [ctypes.c_int32, ctypes.c_int32, dp, dp]
        L.sl_device_field.argtypes = [vp, ctypes.POINTER(vp), ctypes.POINTER(vp)]
        L.sl_set_profiling.argtypes = [vp, ctypes.c_int32]
        L.sl_kernel_time.argtypes = [vp, ctypes.c_int32, dp, ctypes.POINTER(ctypes.c_int64)]
        L.sl_mesh_bytes.argtypes = [ctypes.POINTER(MeshDesc), ctypes.c_int32, ctypes.POINTER(ctypes.c_size_t)]
        L.sl_server_create.argtypes = [ctypes.POINTER(ServerDesc), ctypes.POINTER(vp)]
        L.sl_server_submit.argtypes = [vp, ctypes.POINTER(Request), ctypes.POINTER(ctypes.c_int64)]
        L.sl_server_progress.argtypes = [vp, ctypes.POINTER(ctypes.c_int32), ctypes.POINTER(ctypes.c_int32)]
        L.sl_server_drain.argtypes = [vp]
        L.sl_server_result.argtypes = [vp, ctypes.c_int64, dp, ctypes.POINTER(Stats), ctypes.POINTER(RequestTiming)]
        L.sl_server_latency.argtypes = [vp, dp, ctypes.POINTER(ctypes.c_int64), ctypes.POINTER(ctypes.c_int64)]
        L.sl_server_destroy.argtypes = [vp]
        L.sl_server_batching.argtypes = [vp, ctypes.POINTER(ctypes.c_int64), ctypes.POINTER(ctypes.c_int64)]
        i32, f64 = ctypes.c_int32, ctypes.c_double
        ip = ctypes.POINTER(ctypes.c_int32)
        L.sl_bucket_stats.argtypes = [vp, i32, ip, ip, ip, dp]
        L.sl_step1d_static.argtypes = [i32, i32, i32, i32, i32, f64, f64, vp, vp, vp, vp, f64, vp, f64, i32,
                                       ctypes.POINTER(StepOpts), vp, vp, vp]
        for name in EXPORTS:
            if name not in ("sl_status_string", "sl_max_dt", "sl_ghost_count"):
                getattr(L, name).restype = ctypes.c_int32
        _lib = L
    return _lib


def _dp(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double)) if a is not None else ctypes.POINTER(ctypes.c_double)()


def _f64(a):
    return None if a is None else np.ascontiguousarray(a, dtype=np.float64)


def status_string(s: int) -> str:
    return lib().sl_status_string(int(s)).decode()


def _check(rc: int, where: str):
    if rc != SL_OK:
        raise SLError(rc, where)


# ---- functions named like the C entry points -------------------------------
def sl_node_coords(nodes: int, n: int):
    xi = np.zeros(n)
    w = np.zeros(n)
    _check(lib().sl_node_coords(nodes, n, _dp(xi), _dp(w)), "sl_node_coords")
    return xi, w


def sl_create_mesh(dim, kx, ky, order, u0, nodes=SL_NODES_GL, bc=SL_BC_PERIODIC, form=SL_FORM_ADVECTIVE,
                   precision=SL_PREC_FP64, x0=0.0, x1=1.0, y0=0.0, y1=1.0, stream=None, orders=None):
    """orders: None, or per-element orders N_e (mixed-order 2D mesh)."""
    u0 = _f64(u0)
    od = None if orders is None else np.ascontiguousarray(orders, dtype=np.int32)
    d = MeshDesc(dim, kx, ky, order, nodes, bc, form, precision, x0, x1, y0, y1, _dp(u0),
                 ctypes.c_void_p(stream) if stream else None,
                 od.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)) if od is not None else None)
    h = ctypes.c_void_p()
    _check(lib().sl_create_mesh(ctypes.byref(d), ctypes.byref(h)), "sl_create_mesh")
    return h


def sl_set_velocity(m, a, div_a=None):
    a = _f64(a)
    div_a = _f64(div_a)
    _check(lib().sl_set_velocity(m, _dp(a), _dp(div_a)), "sl_set_velocity")


def sl_set_ghost(m, g, nrows=None):
    g = _f64(g)
    cnt = lib().sl_ghost_count(m)
    nrows = g.size // max(cnt, 1) if nrows is None else nrows
    _check(lib().sl_set_ghost(m, _dp(g), int(nrows)), "sl_set_ghost")


def sl_ghost_count(m) -> int:
    return int(lib().sl_ghost_count(m))


def step_opts(rk=4, constraints=SL_C_BOUNDARY, mode=SL_MODE_HARD, energy_maxit=50, refine_steps=3, energy_tol=1e-8,
              iface=0):
    return StepOpts(rk, constraints, mode, energy_maxit, refine_steps, iface, energy_tol)


def sl_step(m, dt, nsteps=1, opts=None):
    o = opts if opts is not None else step_opts()
    _check(lib().sl_step(m, float(dt), int(nsteps), ctypes.byref(o)), "sl_step")


def sl_step1d_static(K, order, phi_in, phi_out, a, amax, dt, nsteps=1, opts=None, div_a=0, ghost=0,
                     nodes=SL_NODES_GL, bc=SL_BC_PERIODIC, form=SL_FORM_ADVECTIVE, x0=0.0, x1=1.0, stats=0,
                     flags=0, stream=0):
    """1D steps on caller device buffers, allocating nothing (device
    addresses as ints: phi_in, phi_out, a, div_a, ghost, stats, flags)."""
    o = opts if opts is not None else step_opts()
    _check(lib().sl_step1d_static(K, order, nodes, bc, form, x0, x1, phi_in, phi_out, a, div_a or None, amax,
                                  ghost or None, dt, nsteps, ctypes.byref(o), stats or None, flags or None,
                                  stream or None), "sl_step1d_static")


def sl_read(m, size: int):
    """Returns (status, field, Stats); flag statuses are returned, not raised."""
    out = np.zeros(size)
    st = Stats()
    rc = lib().sl_read(m, _dp(out), ctypes.byref(st))
    if rc not in (SL_OK, SL_E_NONFINITE, SL_E_SINGULAR, SL_E_NOCONV):
        raise SLError(rc, "sl_read")
    return rc, out, st


def sl_destroy_mesh(m):
    _check(lib().sl_destroy_mesh(m), "sl_destroy_mesh")


def sl_max_dt(m, cfl=1.0) -> float:
    return float(lib().sl_max_dt(m, float(cfl)))


def sl_device_field(m):
    p = ctypes.c_void_p()
    s = ctypes.c_void_p()
    _check(lib().sl_device_field(m, ctypes.byref(p), ctypes.byref(s)), "sl_device_field")
    return p.value, s.value


def sl_set_profiling(m, enable=True):
    _check(lib().sl_set_profiling(m, 1 if enable else 0), "sl_set_profiling")


def sl_kernel_time(m, which: int):
    ms = ctypes.c_double()
    cnt = ctypes.c_int64()
    _check(lib().sl_kernel_time(m, which, ctypes.byref(ms), ctypes.byref(cnt)), "sl_kernel_time")
    return ms.value, cnt.value


def sl_bucket_stats(m, bucket: int):
    """(n, element count, velocity series terms, mean remap sweeps per element
    and step since the last sl_read) of one order bucket."""
    n, K, vt = ctypes.c_int32(), ctypes.c_int32(), ctypes.c_int32()
    sw = ctypes.c_double()
    _check(lib().sl_bucket_stats(m, int(bucket), ctypes.byref(n), ctypes.byref(K), ctypes.byref(vt),
                                 ctypes.byref(sw)), "sl_bucket_stats")
    return n.value, K.value, vt.value, sw.value


class Mesh:
    """Owns one sl_mesh.  Sizes follow the descriptor; see include/sl.h."""

    def __init__(self, dim, kx, ky, order, u0, **kw):
        self.dim, self.kx, self.ky, self.order = dim, kx, ky, order
        self.n = order + 1
        self.nd = self.n if dim == 1 else self.n * self.n
        self.K = kx * ky
        orders = kw.get("orders")
        self.size = self.K * self.nd if orders is None else int(((np.asarray(orders, dtype=np.int64) + 1) ** 2).sum())
        self.h = sl_create_mesh(dim, kx, ky, order, u0, **kw)

    def set_velocity(self, a, div_a=None):
        sl_set_velocity(self.h, a, div_a)

    def set_ghost(self, g, nrows=None):
        sl_set_ghost(self.h, g, nrows)

    def step(self, dt, nsteps=1, **opts):
        sl_step(self.h, dt, nsteps, step_opts(**opts))

    def read(self):
        return sl_read(self.h, self.size)

    def max_dt(self, cfl=1.0):
        return sl_max_dt(self.h, cfl)

    def close(self):
        if self.h:
            sl_destroy_mesh(self.h)
            self.h = None

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def from_mixed_workload(w, stream=None, precision=SL_PREC_FP64):
    """Mixed-order mesh for a workloads.MixedWorkload, velocity set."""
    m = Mesh(2, w.kx, w.ky, int(w.orders[0]) - 1, w.initial(), nodes=w.family, bc=SL_BC_PERIODIC, form=w.form,
             precision=precision, x0=w.x0, x1=w.x1, y0=w.y0, y1=w.y1, stream=stream,
             orders=np.asarray(w.orders, dtype=np.int32) - 1)
    m.set_velocity(w.velocity())
    return m


def from_workload(w, stream=None, precision=SL_PREC_FP64):
    """Mesh for a workloads.Workload, velocity set (and ghost rows if any)."""
    m = Mesh(w.dim, w.kx, w.ky, w.n - 1, w.initial(), nodes=w.family, bc=w.bc, form=w.form,
             precision=precision, x0=w.x0, x1=w.x1, y0=w.y0, y1=w.y1, stream=stream)
    a, _ = w.velocity()
    m.set_velocity(a)
    return m


def sl_mesh_bytes(dim, kx, ky, order, bc=SL_BC_PERIODIC, ghost_rows=0) -> int:
    d = MeshDesc(dim, kx, ky, order, SL_NODES_GL, bc, SL_FORM_ADVECTIVE, SL_PREC_FP64, 0.0, 1.0, 0.0, 1.0,
                 ctypes.POINTER(ctypes.c_double)(), None)
    b = ctypes.c_size_t()
    _check(lib().sl_mesh_bytes(ctypes.byref(d), int(ghost_rows), ctypes.byref(b)), "sl_mesh_bytes")
    return int(b.value)


class Server:
    """Request loop over the sl_server_* entry points (continuous batching of
    independent problems; see include/sl.h).  Host arrays are copied at
    submission, so the caller's arrays may be reused at once.  The first
    progress() or drain() starts the server's own loop threads; after that
    requests advance without further calls."""

    def __init__(self, max_active=8, hbm_budget=8 << 30, batch=True):
        h = ctypes.c_void_p()
        flags = 0 if batch else SL_SERVER_NO_BATCH
        _check(lib().sl_server_create(ctypes.byref(ServerDesc(int(max_active), flags, int(hbm_budget))),
                                      ctypes.byref(h)), "sl_server_create")
        self.h = h
        self._sizes = {}

    def submit(self, dim, kx, ky, order, u0, a, dt, nsteps, div_a=None, ghost=None, nodes=SL_NODES_GL,
               bc=SL_BC_PERIODIC, form=SL_FORM_ADVECTIVE, precision=SL_PREC_FP64, x0=0.0, x1=1.0, y0=0.0, y1=1.0,
               **opts):
        u0, a, div_a, ghost = _f64(u0), _f64(a), _f64(div_a), _f64(ghost)
        n = order + 1
        nd = n if dim == 1 else n * n
        ng = 2 if dim == 1 else 2 * n * (kx + ky)
        rows = 0 if ghost is None else ghost.size // ng
        mesh = MeshDesc(dim, kx, ky, order, nodes, bc, form, precision, x0, x1, y0, y1, _dp(u0), None)
        req = Request(mesh, _dp(a), _dp(div_a), _dp(ghost), rows, int(nsteps), float(dt), step_opts(**opts))
        rid = ctypes.c_int64()
        _check(lib().sl_server_submit(self.h, ctypes.byref(req), ctypes.byref(rid)), "sl_server_submit")
        self._sizes[rid.value] = kx * ky * nd
        return rid.value

    def progress(self):
        a, w = ctypes.c_int32(), ctypes.c_int32()
        _check(lib().sl_server_progress(self.h, ctypes.byref(a), ctypes.byref(w)), "sl_server_progress")
        return a.value, w.value

    def drain(self):
        _check(lib().sl_server_drain(self.h), "sl_server_drain")

    def result(self, rid):
        """(status, field, Stats, RequestTiming) of a finished request."""
        out = np.zeros(self._sizes.get(rid, 0))
        st, tm = Stats(), RequestTiming()
        rc = lib().sl_server_result(self.h, int(rid), _dp(out), ctypes.byref(st), ctypes.byref(tm))
        if rc == SL_E_STATE or rc == SL_E_INVALID:
            raise SLError(rc, "sl_server_result")
        self._sizes.pop(rid, None)
        return rc, out, st, tm

    def latency(self):
        """(p50 ms, p99 ms, samples, DOF-updates) over retired requests."""
        pp = np.zeros(2)
        n, dof = ctypes.c_int64(), ctypes.c_int64()
        _check(lib().sl_server_latency(self.h, _dp(pp), ctypes.byref(n), ctypes.byref(dof)), "sl_server_latency")
        return float(pp[0]), float(pp[1]), int(n.value), int(dof.value)

    def batching(self):
        """(group steps launched, request steps they carried)."""
        n, m = ctypes.c_int64(), ctypes.c_int64()
        _check(lib().sl_server_batching(self.h, ctypes.byref(n), ctypes.byref(m)), "sl_server_batching")
        return int(n.value), int(m.value)

    def close(self):
        if self.h:
            _check(lib().sl_server_destroy(self.h), "sl_server_destroy")
            self.h = None

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()
