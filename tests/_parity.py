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


def run_gpu(w, phi0=None, nsteps=None, precision=0, ghost=None, div=None, **over):
    """div: nodal divergence handed to the mesh, or None (the derivative of
    the velocity's interpolant, formed on the device)."""
    import paper_1910_06476_amd as P
    nsteps = w.nsteps if nsteps is None else nsteps
    u0 = w.initial() if phi0 is None else phi0
    m = P.Mesh(w.dim, w.kx, w.ky, w.n - 1, u0, nodes=w.family, bc=w.bc, form=w.form, precision=precision,
               x0=w.x0, x1=w.x1, y0=w.y0, y1=w.y1)
    try:
        a, _ = w.velocity()
        m.set_velocity(a, div)
        if w.bc != W.PERIODIC:
            m.set_ghost(w.ghost_rows(0.0, nsteps) if ghost is None else ghost)
        m.step(w.dt, nsteps, **opts_dict(w, **over))
        rc, out, st = m.read()
    finally:
        m.close()
    return out, st, rc


def run_oracle(w, phi0=None, nsteps=None, ghost=None, want=None, div=None, **over):
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
    return oracle.step(p, u0, a=a, div=div, ghost=g, dt=w.dt, nsteps=nsteps, want=want)


def rel_l2(x, ref):
    den = np.linalg.norm(ref)
    return float(np.linalg.norm(x - ref) / (den if den > 0 else 1.0))


def announce(msg):
    """Name the case before each GPU step (flushed), so a fault names it."""
    sys.stdout.write(f"[gpu case] {msg}\n")
    sys.stdout.flush()


def assert_parity(w, g, o, tol=1e-12, elems=None):
    """GPU-vs-oracle parity on the whole field (or on the elements `elems`):
    relative L2 <= tol, and no value off by more than 10 tol of the largest
    magnitude.  Returns the relative L2."""
    G = np.asarray(g).reshape(w.K, w.nd)
    O = np.asarray(o).reshape(w.K, w.nd)
    if elems is not None:
        G, O = G[elems], O[elems]
    err = rel_l2(G, O)
    assert err <= tol, f"rel L2 {err:.3e} > {tol:.0e}"
    scale = max(float(np.abs(O).max()), 1e-300)
    worst = float(np.abs(G - O).max()) / scale
    assert worst <= 10 * tol, f"max abs error {worst:.3e} of max |o| > {10 * tol:.0e}"
    return err
