"""Helpers for GPU-vs-oracle parity tests: run one workload through the
C-ABI (HIP path) and through the oracle on identical seeded inputs."""
import sys

import numpy as np

import oracle
import workloads as W


def opts_dict(w, **over):
    d = dict(rk=w.rk, constraints=w.cmask, mode=w.mode, energy_maxit=w.energy_maxit,
             energy_tol=w.energy_tol, refine_steps=3)
    d.update(over)
    return d


def run_gpu(w, phi0=None, nsteps=None, precision=0, ghost=None, **over):
    import paper_1910_06476_amd as P
    nsteps = w.nsteps if nsteps is None else nsteps
    u0 = w.initial() if phi0 is None else phi0
    m = P.Mesh(w.dim, w.kx, w.ky, w.n - 1, u0, nodes=w.family, bc=w.bc, form=w.form, precision=precision,
               x0=w.x0, x1=w.x1, y0=w.y0, y1=w.y1)
    try:
        a, _ = w.velocity()
        m.set_velocity(a)
        if w.bc != W.PERIODIC:
            m.set_ghost(w.ghost_rows(0.0, nsteps) if ghost is None else ghost)
        m.step(w.dt, nsteps, **opts_dict(w, **over))
        rc, out, st = m.read()
    finally:
        m.close()
    return out, st, rc


def run_oracle(w, phi0=None, nsteps=None, ghost=None, want=None, **over):
    nsteps = w.nsteps if nsteps is None else nsteps
    u0 = w.initial() if phi0 is None else phi0
    kw = {}
    if "energy_maxit" in over:
        kw["energy_maxit"] = over.pop("energy_maxit")
    if "energy_tol" in over:
        kw["energy_tol"] = over.pop("energy_tol")
    if "rk" in over:
        kw["rk"] = over.pop("rk")
    if "constraints" in over:
        kw["cmask"] = over.pop("constraints")
    if "mode" in over:
        kw["mode"] = over.pop("mode")
    if "iface" in over:
        kw["iface"] = over.pop("iface")
    over.pop("refine_steps", None)
    p = oracle.params_from(w, **kw)
    a, _ = w.velocity()
    g = None
    if w.bc != W.PERIODIC:
        g = w.ghost_rows(0.0, nsteps) if ghost is None else ghost
    return oracle.step(p, u0, a=a, ghost=g, dt=w.dt, nsteps=nsteps, want=want)


def rel_l2(x, ref):
    den = np.linalg.norm(ref)
    return float(np.linalg.norm(x - ref) / (den if den > 0 else 1.0))


def announce(msg):
    """Name the case before each GPU step (flushed), so a fault names it."""
    sys.stdout.write(f"[gpu case] {msg}\n")
    sys.stdout.flush()


EPS = np.finfo(np.float64).eps


def energy_kappa(w, phi):
    """Per-element amplification of rounding by a HARD energy row: 1/sin of
    the angle between the energy row W*phi and the mass row W,
    kappa_e = |W*phi|_2 / |W*phi - mu W|_2 (mu = projection coefficient).
    A result constrained by both rows is determined in FP64 only to about
    eps * kappa_e relative to the element's values."""
    xi, wq = oracle.nodes(w.family, w.n)
    if w.dim == 1:
        Wr = wq * w.dx
    else:
        Wr = np.outer(wq, wq).ravel() * w.dx * w.dy
    P = np.asarray(phi).reshape(w.K, w.nd)
    g = Wr * P
    mu = (g @ Wr) / (Wr @ Wr)
    gp = g - mu[:, None] * Wr
    return np.linalg.norm(g, axis=1) / np.maximum(np.linalg.norm(gp, axis=1), 1e-300)


def assert_parity(w, g, o, cmask=None, mode=None, tol=1e-12, elems=None, solves=None):
    """GPU-vs-oracle parity.  Without a HARD energy row: relative L2 <= tol.
    With one (and a mass row) each energy-constrained solve is exact only to
    about eps * kappa_e, and these errors add up over the Picard sweeps and
    the steps (the sweep map has an eigenvalue near -1, so they are neither
    damped nor amplified); element-wise bound
    |g_e - o_e|_max <= max(tol, 64 eps kappa_e * solves) |o_e|_max,
    solves = steps * sweeps (default from the workload)."""
    cmask = w.cmask if cmask is None else cmask
    mode = w.mode if mode is None else mode
    G = np.asarray(g).reshape(w.K, w.nd)
    O = np.asarray(o).reshape(w.K, w.nd)
    if elems is not None:
        G, O = G[elems], O[elems]
    hard_e = (cmask & W.ENERGY) and (cmask & W.MASS) and mode == W.HARD
    if not hard_e:
        err = rel_l2(G, O)
        assert err <= tol, f"rel L2 {err:.3e} > {tol:.0e}"
        return err
    k = energy_kappa(w, o)
    if elems is not None:
        k = k[elems]
    if solves is None:
        solves = max(1, w.nsteps) * max(1, w.energy_maxit)
    bound = np.maximum(tol, 64 * EPS * k * solves) * np.maximum(np.abs(O).max(1), 1e-300)
    e = np.abs(G - O).max(1)
    bad = np.nonzero(e > bound)[0]
    assert bad.size == 0, f"{bad.size} elements above the conditioning bound, worst ratio {np.max(e / bound):.2f}"
    return rel_l2(G, O)
