"""CPU oracle for the explicit semi-Lagrangian spectral step (FP64).

TEST INFRASTRUCTURE ONLY: the test-suite, the smoke check and the benchmark's
``cpu_baseline`` leg may import this package; the product path never does.
It wraps ``sl_oracle.c`` (plain C, OpenMP over elements), which shares no code
with the HIP library.  Each entry point follows a passage of the paper
(Natarajan & Jacobs, arXiv 1910.06476), cited in the C source.

Parity pins: every function here is pinned by ``tests/test_oracle_*.py``
against closed forms, library routines, brute force and the paper's printed
Tables 2 and 3 (see the test docstrings).  Pieces without such a pin are
marked "parity unpinned" where they are defined.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "sl_oracle.c")
_LIB = os.environ.get("SL_ORACLE_LIB") or os.path.join(_HERE, "liboracle.so")


def build(force: bool = True) -> str:
    """Compile the oracle (gcc -O2, OpenMP, no fast-math)."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp"
        subprocess.check_call(
            ["gcc", "-O2", "-std=c11", "-fopenmp", "-fPIC", "-shared", "-D_DEFAULT_SOURCE",
             "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


def use_native_build() -> str:
    """Compile the oracle with -O3 -march=native (still no fast-math) for the
    host this process runs on, into a temporary directory, and load that
    build from now on.  Used by the benchmark's CPU baseline: the machine
    code is the host's own, so the build happens where it is timed."""
    global _LIB, _lib
    import tempfile
    out = os.path.join(tempfile.mkdtemp(prefix="sl_oracle_"), "liboracle_native.so")
    subprocess.check_call(
        ["gcc", "-O3", "-march=native", "-std=c11", "-fopenmp", "-fPIC", "-shared", "-D_DEFAULT_SOURCE",
         "-o", out, _SRC, "-lm"])
    _LIB, _lib = out, None
    return out


class Params(ctypes.Structure):
    _fields_ = [
        ("dim", ctypes.c_int32), ("kx", ctypes.c_int32), ("ky", ctypes.c_int32),
        ("n", ctypes.c_int32), ("family", ctypes.c_int32), ("bc", ctypes.c_int32),
        ("form", ctypes.c_int32), ("rk", ctypes.c_int32), ("cmask", ctypes.c_int32),
        ("mode", ctypes.c_int32), ("energy_maxit", ctypes.c_int32), ("vel_kind", ctypes.c_int32),
        ("x0", ctypes.c_double), ("x1", ctypes.c_double), ("y0", ctypes.c_double),
        ("y1", ctypes.c_double), ("energy_tol", ctypes.c_double),
        ("vel_param", ctypes.c_double * 4), ("iface", ctypes.c_int32),
    ]


class Stats(ctypes.Structure):
    _fields_ = [
        ("resid_boundary", ctypes.c_double), ("resid_mass", ctypes.c_double),
        ("resid_energy", ctypes.c_double), ("max_picard", ctypes.c_int32),
        ("flags", ctypes.c_int32),
    ]

    def asdict(self):
        return {f: getattr(self, f) for f, _ in self._fields_}


F_NONFINITE, F_CONTAIN, F_SINGULAR, F_NOCONV = 1, 2, 4, 8

_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build(force=False)
        L = ctypes.CDLL(_LIB)
        dp = ctypes.POINTER(ctypes.c_double)
        L.ora_nodes.argtypes = [ctypes.c_int, ctypes.c_int, dp, dp]
        L.ora_lagrange.argtypes = [ctypes.c_int, dp, ctypes.c_double, dp]
        L.ora_ghost_count.argtypes = [ctypes.POINTER(Params)]
        L.ora_step_mixed.argtypes = [ctypes.POINTER(Params), ctypes.POINTER(ctypes.c_int32), dp, ctypes.c_double,
                                     ctypes.c_int, dp, ctypes.POINTER(Stats)]
        L.ora_step.argtypes = [ctypes.POINTER(Params), dp, dp, dp, ctypes.c_int, ctypes.c_double,
                               ctypes.c_int, dp, ctypes.POINTER(ctypes.c_uint8), ctypes.POINTER(Stats)]
        L.ora_rk_tableau.argtypes = [ctypes.c_int, ctypes.POINTER(ctypes.c_int), dp, dp, dp]
        L.ora_cls.argtypes = [ctypes.c_int, ctypes.c_int, dp, dp, dp, ctypes.c_int, dp]
        L.ora_boundary_pinv.argtypes = [ctypes.c_int, ctypes.c_int, dp, dp]
        L.ora_energy_hard.argtypes = [ctypes.c_int, ctypes.c_int, dp, dp, dp, ctypes.c_double, ctypes.c_double,
                                      dp, ctypes.c_double, ctypes.c_int, dp, ctypes.POINTER(ctypes.c_int)]
        _lib = L
    return _lib


def _p(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def nodes(family: int, n: int):
    """Reference nodes and weights on [0,1] (section 3, eq. gaussquad for
    Chebyshev-Gauss; Gauss-Legendre by Newton on the Legendre recurrence)."""
    xi = np.zeros(n)
    w = np.zeros(n)
    if lib().ora_nodes(family, n, _p(xi), _p(w)):
        raise ValueError("bad node family/count")
    return xi, w


def lagrange(x, t):
    """Lagrange basis on nodes x at t, product form (eq. 3.5)."""
    x = np.ascontiguousarray(x, dtype=np.float64)
    out = np.zeros(len(x))
    lib().ora_lagrange(len(x), _p(x), float(t), _p(out))
    return out


def rk_tableau(rk: int):
    s = ctypes.c_int()
    a = np.zeros(16)
    b = np.zeros(4)
    c = np.zeros(4)
    if lib().ora_rk_tableau(rk, ctypes.byref(s), _p(a), _p(b), _p(c)):
        raise ValueError(rk)
    return s.value, a.reshape(4, 4), b, c


def cls(C, d, phihat, mode: int):
    """Constrained least squares of eq. matrix_a: HARD (mode 0) imposes
    C phi = d exactly with minimal ||phi - phihat||; SOFT (mode 1) minimises
    ||phi - phihat||^2 + ||C phi - d||^2."""
    C = np.ascontiguousarray(C, dtype=np.float64)
    d = np.ascontiguousarray(d, dtype=np.float64)
    ph = np.ascontiguousarray(phihat, dtype=np.float64)
    out = np.zeros(len(ph))
    bad = lib().ora_cls(len(ph), C.shape[0], _p(C), _p(d), _p(ph), mode, _p(out))
    if bad:
        raise np.linalg.LinAlgError("singular constrained system")
    return out


def energy_hard(C, d, Wq, s, T, phihat, tol=0.0, maxit=20):
    """HARD constrained least squares with the energy row as the step imposes
    it (section "Local energy conservation", eq. remap_energy, with the
    reading of its fixed-point iteration documented in sl_oracle.c):
    min ||phi - phihat|| s.t. C phi = d and sum Wq (phi - s)^2 = T.
    Returns (phi, sweeps, flags)."""
    C = np.ascontiguousarray(np.atleast_2d(C), dtype=np.float64)
    d = np.ascontiguousarray(d, dtype=np.float64)
    Wq = np.ascontiguousarray(Wq, dtype=np.float64)
    ph = np.ascontiguousarray(phihat, dtype=np.float64)
    out = np.zeros(len(ph))
    fl = ctypes.c_int()
    m = C.shape[0] if C.size else 0
    k = lib().ora_energy_hard(len(ph), m, _p(C), _p(d), _p(Wq), float(s), float(T), _p(ph), float(tol),
                              int(maxit), _p(out), ctypes.byref(fl))
    return out, k, fl.value


def boundary_pinv(family: int, n: int):
    CB = np.zeros((4 * n, n * n))
    CBp = np.zeros((n * n, 4 * n))
    lib().ora_boundary_pinv(family, n, _p(CB), _p(CBp))
    return CB, CBp


def params_from(w, **over) -> Params:
    """Parameter block from a workloads.Workload (keyword overrides allowed)."""
    p = Params()
    fields = dict(dim=w.dim, kx=w.kx, ky=w.ky, n=w.n, family=w.family, bc=w.bc, form=w.form,
                  rk=w.rk, cmask=w.cmask, mode=w.mode, energy_maxit=w.energy_maxit, vel_kind=0,
                  x0=w.x0, x1=w.x1, y0=w.y0, y1=w.y1, energy_tol=w.energy_tol)
    fields.update(over)
    vp = fields.pop("vel_param", None)
    for k, v in fields.items():
        setattr(p, k, v)
    if vp is not None:
        for i, v in enumerate(vp):
            p.vel_param[i] = v
    return p


def step(p: Params, phi, a=None, div=None, ghost=None, dt=0.0, nsteps=1, want=None):
    """Advance phi by nsteps explicit SL steps of length dt.

    a: nodal velocity [dim][K][nd] (ignored for analytic velocity kinds);
    div: nodal divergence [K][nd] or None (derivative of the interpolant);
    ghost: [rows][nghost] inflow values (row i used at step i, last row
    repeated); want: optional element mask (single step only).
    Returns (phi_out, Stats)."""
    phi = np.array(phi, dtype=np.float64, copy=True)
    nd = p.n if p.dim == 1 else p.n * p.n
    K = p.kx * p.ky
    if phi.size != K * nd:
        raise ValueError("phi has the wrong size")
    nullp = ctypes.POINTER(ctypes.c_double)()
    a_ = np.ascontiguousarray(a, dtype=np.float64) if a is not None else None
    if p.vel_kind == 0 and (a_ is None or a_.size != p.dim * K * nd):
        raise ValueError("nodal velocity required")
    d_ = np.ascontiguousarray(div, dtype=np.float64) if div is not None else None
    g_ = None
    rows = 0
    if ghost is not None:
        g_ = np.ascontiguousarray(ghost, dtype=np.float64)
        ng = lib().ora_ghost_count(ctypes.byref(p))
        if g_.size % ng:
            raise ValueError("ghost array has the wrong size")
        rows = g_.size // ng
    m_ = None
    if want is not None:
        m_ = np.ascontiguousarray(want, dtype=np.uint8)
    st = Stats()
    rc = lib().ora_step(ctypes.byref(p), _p(a_) if a_ is not None else nullp,
                        _p(d_) if d_ is not None else nullp,
                        _p(g_) if g_ is not None else nullp, rows, float(dt), int(nsteps), _p(phi),
                        m_.ctypes.data_as(ctypes.POINTER(ctypes.c_uint8)) if m_ is not None else
                        ctypes.POINTER(ctypes.c_uint8)(), ctypes.byref(st))
    if rc:
        raise ValueError("oracle rejected the parameters")
    return phi, st


def run_workload(w, nsteps=None, analytic=False, ghost_t0=0.0, **over):
    """Run a workloads.Workload from its initial field on the oracle."""
    nsteps = w.nsteps if nsteps is None else nsteps
    kw = dict(over)
    if analytic:
        kw["vel_kind"] = w.vel_kind
        if w.vel_kind == 1:
            x, y = w.coords()
            u, v, _ = w.vel(x, y)
            kw["vel_param"] = [float(np.ravel(u)[0]), float(np.ravel(v)[0]) if np.ndim(v) else float(v), 0, 0]
    p = params_from(w, **kw)
    a, _ = w.velocity()
    ghost = w.ghost_rows(ghost_t0, nsteps) if w.bc != 0 else None
    return step(p, w.initial(), a=a, ghost=ghost, dt=w.dt, nsteps=nsteps)


def step_mixed(p: Params, orders, phi, a=None, dt=0.0, nsteps=1):
    """Mixed-order 2D step (periodic, boundary rows): orders[K] nodes per
    direction per element; phi and each velocity component concatenated
    element by element (n_e^2 values each); a = u values then v values."""
    orders = np.ascontiguousarray(orders, dtype=np.int32)
    phi = np.array(phi, dtype=np.float64, copy=True)
    if phi.size != int((orders.astype(np.int64) ** 2).sum()):
        raise ValueError("phi has the wrong size")
    nullp = ctypes.POINTER(ctypes.c_double)()
    a_ = None if a is None else np.ascontiguousarray(a, dtype=np.float64)
    if p.vel_kind == 0 and (a_ is None or a_.size != 2 * phi.size):
        raise ValueError("nodal velocity required")
    st = Stats()
    rc = lib().ora_step_mixed(ctypes.byref(p), orders.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)),
                              _p(a_) if a_ is not None else nullp, float(dt), int(nsteps), _p(phi), ctypes.byref(st))
    if rc:
        raise ValueError("oracle rejected the parameters")
    return phi, st
