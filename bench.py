"""Benchmark of the explicit semi-Lagrangian spectral step on one MI355X.

Workload of the headline line (the largest configuration on one GPU): the
2D mixed-order batch, 316 x 316 quads on [0,1]^2 (8.08 M DOF) with the order
of each element drawn from {4, 6, 8, 12} by seed, the swirl velocity
a = (sin^2(pi x) sin(2 pi y), -sin^2(pi y) sin(2 pi x)), eight random Fourier
modes, periodic, boundary rows (HARD), RK4, FP64.  One "step" is one sl_step
over the whole mesh (every order bucket, all stages of the method), replayed
from the mesh's captured graph.  Inputs are resident in HBM before the timed
region.

Prints one JSON line: DOF-updates/s over K timed steps, the stated L2 error
(here of a forward-and-back round trip under the steady swirl, whose exact
result is the initial field), the served per-step latency (p50/p99), the
roofline of the dominant kernel (HIP events on the mesh's stream around
every launch, algorithmic flop count per element from the functions below),
and the CPU oracle timed on a bounded sample.  Other workloads: --workload
c2 (the 1D configuration with boundary, mass and energy rows), c3 (2D
rotation, --precision fp64 / fp32r / bf16r, --constraints b / bm / bme),
c2bw (HBM probe), c1 (launch latency), serve (a Poisson stream of
independent problems through the request loop).
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "DOF-updates/sec per sl_step at stated L2 error; served p50/p99 step latency"
FP64_VALU_PEAK = 78.6e12   # 256 CU x 4 SIMD x 16 lanes x 2 flop x 2.4 GHz (FMA = 2 flops)
HBM_PEAK = 8.0e12


def advect_flops_per_element(n: int, s: int, nq: int, targets: bool, vel_terms: int) -> float:
    """Algorithmic FP64 flops of the 1D advect kernel for one element (FMA = 2):
    velocity series of at most 4 terms by Horner's rule on its polynomial in
    the element coordinate (2 flops per term after the first), longer ones
    and phi^n by Clenshaw (3 flops per term); RK stage update ~4 flops per
    stage; remap in product form (5 flops per node and point)."""
    clen = 3.0 * n
    clen_v = 2.0 * (vel_terms - 1) if vel_terms <= 4 else 3.0 * vel_terms
    rk_move = (s - 1) * clen_v + 4.0 * s
    f = n * rk_move                      # forward motion of the n particles
    f += n * (2.0 * n)                   # moved-point weights lambda*: n-1 (sub, mul) + div
    f += n * (5.0 * n) + 5.0 * n         # remap at n nodes and at 0 (product form)
    f += 3.0 * n                         # trace at 1: l(1) . phihat
    if targets:
        f += 2.0 * n * n                 # Chebyshev coefficients of phi^n
        back = rk_move + clen            # one backtrace + evaluation of phi^n at its foot
        f += n * (nq - 1) * (back + 6)   # node backtraces (volume term)
        f += 2 * ((nq - 1) * (back + 4) + n)  # edge values at the RK abscissae (at t^n: end-point sum)
        f += 8.0 * n                     # mass/energy sums
    return f


def advect_bytes_per_element(n: int, targets: bool, vel_terms: int) -> float:
    """Algorithmic HBM bytes of the 1D advect kernel per element: read phi^n
    and the nodal velocity (+ the nodal divergence and the face speed with
    targets) and the velocity series coefficients that are evaluated; write
    phihat and the element record (the two traces, + the six target entries
    and the element's mean with targets)."""
    rd = 8.0 * n * (3 if targets else 2) + 8.0 * vel_terms + (8.0 if targets else 0.0)
    wr = 8.0 * n + (72.0 if targets else 16.0)
    return rd + wr


def constrain_bytes_per_element(n: int, targets: bool = True) -> float:
    """read phihat, the element record entries in use (the two traces, + the
    targets' six and the element's mean; the neighbours' are cache hits) and
    one face speed; write phi."""
    return 8.0 * n + (72.0 if targets else 16.0) + 8.0 + 8.0 * n


def measured_traffic(kernel: str, source: str = "sl1d.hip", profile: str = "sl1d_c2_K65536_n17.md"):
    """HBM bytes per launch from the committed rocprofv3 FETCH_SIZE/WRITE_SIZE
    summary, or None if the kernel source changed since it was taken."""
    import hashlib
    src = os.path.join(ROOT, "paper_1910_06476_amd", "csrc", source)
    sha = hashlib.sha256(open(src, "rb").read()).hexdigest()[:16]
    path = os.path.join(ROOT, "profiles", profile)
    if not os.path.exists(path):
        return None
    for line in open(path):
        parts = line.split()
        if len(parts) == 4 and parts[0] == "traffic" and parts[1] == kernel and parts[3] == f"{source}:{sha}":
            return float(parts[2])
    return None


def host_cpu():
    """The host's CPU model and logical CPU count, printed with the oracle
    baseline."""
    model = "unknown"
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    return {"cpu_model": model, "nproc": os.cpu_count()}


def single_thread_rate(run, dofs: int, est_s: float, limit_s: float = 15.0):
    """DOF-updates/s of one oracle step on one OpenMP thread (the OpenMP
    runtime's thread count is set to 1 and restored); None when that step
    would take longer than limit_s (est_s: the all-core step time times the
    thread count) or the runtime cannot be reached."""
    import ctypes
    if est_s > limit_s:
        return None
    try:
        gomp = ctypes.CDLL("libgomp.so.1")
    except OSError:
        return None
    prev = gomp.omp_get_max_threads()
    gomp.omp_set_num_threads(1)
    try:
        t0 = time.perf_counter()
        run()
        return dofs / (time.perf_counter() - t0)
    finally:
        gomp.omp_set_num_threads(prev)


def native_oracle():
    """The oracle built with -O3 -march=native on this host (once)."""
    import oracle
    if not getattr(native_oracle, "done", False):
        oracle.use_native_build()
        native_oracle.done = True
    return oracle


def cpu_baseline(w, budget_s: float = 12.0, div=None):
    """The oracle on the full mesh of `w` (div: the nodal divergence the
    device was given, else None for the interpolant's)."""
    import workloads as W
    oracle = native_oracle()
    p = oracle.params_from(w)
    a, _ = w.velocity()
    phi = w.initial()
    ghost = w.bc != W.PERIODIC  # inflow rows from the exact solution, as on the device
    t0 = time.perf_counter()
    phi, _ = oracle.step(p, phi, a=a, div=div, ghost=w.ghost_rows(0.0, 1) if ghost else None, dt=w.dt, nsteps=1)
    one = time.perf_counter() - t0
    steps = max(1, min(50, int(budget_s / max(one, 1e-3))))
    g = w.ghost_rows(w.dt, steps) if ghost else None
    t0 = time.perf_counter()
    oracle.step(p, phi, a=a, div=div, ghost=g, dt=w.dt, nsteps=steps)
    el = time.perf_counter() - t0
    cores = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    g1 = w.ghost_rows(0.0, 1) if ghost else None
    one_thread = single_thread_rate(lambda: oracle.step(p, phi, a=a, div=div, ghost=g1, dt=w.dt, nsteps=1), w.dofs,
                                    el / steps * cores)
    return {"value": w.dofs * steps / el, "unit": "DOF-updates/s", "cores": cores, "kind": "oracle",
            "single_thread_value": one_thread,
            "sample": f"full mesh (K={w.K}, n={w.n}), {steps} steps after 1 warm-up step, "
                      f"{el:.1f} s, OpenMP threads={cores}, gcc -O3 -march=native", **host_cpu()}


def cpu_baseline_mixed(w, budget_s: float = 12.0):
    """The mixed-order oracle on `w` (a piece of the C4 recipe), timed over
    as many steps as fit in about budget_s."""
    import workloads as W
    oracle = native_oracle()
    p = oracle.Params(dim=2, kx=w.kx, ky=w.ky, n=int(w.orders[0]), family=w.family, bc=W.PERIODIC, form=w.form,
                      rk=w.rk, cmask=W.BOUNDARY, mode=w.mode, energy_maxit=0, vel_kind=0, x0=w.x0, x1=w.x1,
                      y0=w.y0, y1=w.y1, energy_tol=0.0)
    a = w.velocity()
    phi, _ = oracle.step_mixed(p, w.orders, w.initial(), a=a, dt=w.dt, nsteps=1)
    # every call first builds the per-element tables: size the sample from
    # the marginal cost of a step (calls of 1 and 5 steps), so that the
    # tables take a small part of it
    t0 = time.perf_counter()
    oracle.step_mixed(p, w.orders, phi, a=a, dt=w.dt, nsteps=1)
    t1 = time.perf_counter()
    oracle.step_mixed(p, w.orders, phi, a=a, dt=w.dt, nsteps=5)
    t5 = time.perf_counter() - t1
    t1 -= t0
    per = max((t5 - t1) / 4, 1e-4)
    setup = max(t1 - per, 0.0)
    steps = max(1, min(2000, int(max(budget_s - setup, per) / per)))
    t0 = time.perf_counter()
    oracle.step_mixed(p, w.orders, phi, a=a, dt=w.dt, nsteps=steps)
    el = time.perf_counter() - t0
    cores = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    # one thread: a call of k1 steps, about 4 s of stepping, set-up included
    k1 = max(1, min(steps, int(4.0 / (per * cores))))
    one_thread = single_thread_rate(lambda: oracle.step_mixed(p, w.orders, phi, a=a, dt=w.dt, nsteps=k1),
                                    w.dofs * k1, setup + k1 * per * cores)
    return {"value": w.dofs * steps / el, "unit": "DOF-updates/s", "cores": cores, "kind": "oracle",
            "single_thread_value": one_thread,
            "sample": f"a {w.kx}x{w.ky} mesh of the same recipe (orders {{4,6,8,12}} by seed, {w.dofs} DOF), "
                      f"{steps} steps in one call after 3 warm-up calls, {el:.1f} s (the call's table set-up, "
                      f"about {setup:.1f} s, included), OpenMP threads={cores}, gcc -O3 -march=native", **host_cpu()}


def advect2d_flops_per_element(n: int, s: int, sweeps: float, vel_terms: int) -> float:
    """Algorithmic FP64 flops of the 2D advect+solve kernel per element:
    motion (the tensor Chebyshev series summed directly over T_k(x) T_l(y),
    one FMA per coefficient: 2 m^2 flops per component, 2 components, plus
    the T recurrences, 8 (m - 2) for m > 2; (s-1) evaluations per particle),
    the V rows (product form, ~6n per particle), the separable preconditioner
    (2 n^2 (n-1) products to build, 4 n^3 per application), and per
    defect-correction sweep the matrix-free V x (2 n^4 + 2 n^2) plus one
    preconditioner application."""
    nd = n * n
    m = vel_terms
    ev = 2 * 2.0 * m * m + 8.0 * max(m - 2, 0)
    f = nd * ((s - 1) * ev + 8.0 * s)
    f += nd * 6.0 * n
    f += 2 * nd * 4.0 * (n - 1)
    apply = 4.0 * n ** 3
    f += apply
    f += sweeps * (2.0 * n ** 4 + 2.0 * nd + apply + 2.0 * nd)
    f += 4 * n * 2.0 * n
    return f


def step_latency(torch, m, dt, opts, samples=200):
    """Served per-step latency: one sl_step submitted and waited for at a
    time (host validation, both launches and the synchronisation), as a
    request loop sees it; p50 and p99 over `samples` steps, microseconds."""
    lat = []
    for _ in range(samples):
        t0 = time.perf_counter()
        m.step(dt, 1, **opts)
        torch.cuda.synchronize()
        lat.append((time.perf_counter() - t0) * 1e6)
    lat.sort()
    pick = lambda q: lat[min(len(lat) - 1, int(q * len(lat)))]
    return {"p50_us": pick(0.50), "p99_us": pick(0.99), "samples": samples}


def profiled_window(P, m, dt, nsteps, opts, kinds, acc=None):
    """Run nsteps steps with per-kernel timing: each launch of a kernel in
    `kinds` is timed by the start and end its own dispatch records (the
    interval a kernel trace reports).  Adds (total ms, launches) per kind to
    acc.

    The device's clocks drift within a run: they rise from idle over the
    first few hundred launches and fall under sustained FP64 load.  The bench
    lines therefore time one window just before the timed region and one of
    the same length just after it; with a drift close to linear over the
    timed region, their pooled average is the timed region's."""
    acc = {} if acc is None else acc
    P.sl_set_profiling(m.h, True)
    m.step(dt, nsteps, **opts)
    for k in kinds:
        t, c = P.sl_kernel_time(m.h, k)
        a = acc.get(k, (0.0, 0))
        acc[k] = (a[0] + t, a[1] + c)
    P.sl_set_profiling(m.h, False)
    return acc


def avg_us(acc, k):
    t, c = acc[k]
    return t / max(c, 1) * 1e3


C3_ROWS = {"b": ("boundary HARD", "B"), "bm": ("boundary+mass HARD", "B+M"),
           "bme": ("boundary+mass+energy HARD, energy stop 1e-8", "B+M+E")}


def bench_c3(args, torch, P, W, stream):
    """2D rotation workload (256x256, order 8, RK4, ghost inflow), boundary
    rows HARD, or with --constraints bm / bme also the mass (and energy)
    rows: their targets kernel backtraces phi^n from the upwind edge points
    (and from every node where the divergence is nonzero).  The mesh gets
    the flow's exact divergence, zero."""
    w = W.c3(nsteps=args.warmup + args.steps)
    w.cmask = {"b": W.BOUNDARY, "bm": W.BOUNDARY | W.MASS, "bme": W.BOUNDARY | W.MASS | W.ENERGY}[args.constraints]
    prec = {"fp64": P.SL_PREC_FP64, "fp32r": P.SL_PREC_FP32_REFINED, "bf16r": P.SL_PREC_BF16_REFINED}[args.precision]
    m = P.from_workload(w, stream=stream.cuda_stream, precision=prec)
    a, div = w.velocity()
    m.set_velocity(a, div)
    targets = args.constraints != "b"
    nprof = max(5, min(args.steps, 20))
    nlat = min(100, max(10, args.steps))
    # inflow rows for every step the run takes (and one more time level)
    m.set_ghost(w.ghost_rows(0.0, args.warmup + args.steps + 2 * nprof + nlat + 2))
    opts = dict(rk=w.rk, constraints=w.cmask, mode=w.mode, energy_maxit=w.energy_maxit, energy_tol=w.energy_tol)
    m.step(w.dt, args.warmup, **opts)
    kinds = [P.KER_ADV2D, P.KER_CON2D] + ([P.KER_TGT2D] if targets else [])
    acc = profiled_window(P, m, w.dt, nprof, opts, kinds)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    m.step(w.dt, args.steps, **opts)
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    profiled_window(P, m, w.dt, nprof, opts, kinds, acc)
    rc, phi, st = m.read()
    T = st.t
    l2 = w.l2_error(phi, T)
    sweeps = st.remap_sweeps_mean  # defect-correction sweeps per element and step, measured
    lat = step_latency(torch, m, w.dt, opts, samples=nlat)
    m.close()
    adv_avg = avg_us(acc, P.KER_ADV2D) * 1e-6
    con_avg = avg_us(acc, P.KER_CON2D) * 1e-6
    fl = advect2d_flops_per_element(w.n, 4, sweeps, st.vel_terms) * w.K
    ach = fl / adv_avg
    out = {
        "metric": METRIC, "value": w.dofs * args.steps / el, "unit": "DOF-updates/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": el / args.steps * 1e3,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f64", "data": "synthetic",
        "config": {"workload": "2D rotation a=(-(y-1/2),x-1/2) on [0,1]^2, 256x256, order 8 (81 nodes/elem), "
                               "Gaussian hill, RK4, ghost inflow from the exact solution, " + C3_ROWS[args.constraints][0],
                   "K": w.K, "n": w.n, "dofs": w.dofs, "dt": w.dt, "constraints": C3_ROWS[args.constraints][1],
                   "divergence": "exact (zero)"},
        "l2_error": l2, "l2_time": T, "status": P.status_string(rc), "precision": args.precision,
        "step_latency": lat,
        "remap_sweeps_mean": sweeps, "remap_sweeps_max": st.remap_sweeps_max, "refine_resid": st.refine_resid,
        "vel_terms": st.vel_terms,
        "roofline": {"kernel": "sl2d_advect", "bound": "alu", "achieved": ach / 1e12,
                     "peak": FP64_VALU_PEAK / 1e12, "unit": "TFLOP/s", "frac": ach / FP64_VALU_PEAK,
                     "traffic": measured_traffic("k_advect2d", "sl2d_kernels.h", "sl2d_c3_256x256_n9.md")
                     if args.precision == "fp64" and not targets else None,
                     "avg_launch_us": adv_avg * 1e6, "algorithmic_flops_per_launch": fl,
                     "kernels_us": {"sl2d_advect": adv_avg * 1e6, "sl2d_constrain": con_avg * 1e6}},
    }
    if targets:
        out["roofline"]["kernels_us"]["sl2d_targets"] = avg_us(acc, P.KER_TGT2D)
        out["max_picard"] = st.max_picard
    if not args.no_cpu:
        out["cpu_baseline"] = cpu_baseline(w, div=div)
    print(json.dumps(out))


def bench_c4(args, torch, P, W, stream):
    """Mixed-order batch: 316 x 316 quads, per-element order drawn from
    {4, 6, 8, 12} by seed, swirl velocity, eight Fourier modes, periodic,
    boundary rows (HARD), RK4, dt = 2.107e-5.  Order buckets run as
    separate launches captured in one HIP graph per two steps, with the
    advect block shape per bucket picked by the autotuner at the first step.

    Stated error: 100 steps forward, the velocity reversed, 100 steps back;
    the exact result of that round trip is the initial field, and the L2
    norm of the difference (the paper's norm, eq. 5.2) is the scheme's error
    over 200 steps."""
    prec = {"fp64": P.SL_PREC_FP64, "fp32r": P.SL_PREC_FP32_REFINED, "bf16r": P.SL_PREC_BF16_REFINED}[args.precision]
    w = W.c4(nsteps=args.warmup + args.steps)
    m = P.from_mixed_workload(w, stream=stream.cuda_stream, precision=prec)
    opts = dict(rk=w.rk, constraints=W.BOUNDARY, mode=w.mode)
    m.step(w.dt, max(2, args.warmup), **opts)  # autotune, capture, warm up
    nb = len(set(w.orders.tolist()))
    kinds = [P.KER_ADV2D] + [P.KER_MIX_ADV + b for b in range(nb)] + [P.KER_MIX_CON + b for b in range(nb)]
    # per-kernel timing around the timed region (the profiled steps run the
    # graph's launches one by one)
    nprof = max(4, min(args.steps, 20))
    acc = profiled_window(P, m, w.dt, nprof, opts, kinds)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    m.step(w.dt, args.steps, **opts)
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    profiled_window(P, m, w.dt, nprof, opts, kinds, acc)
    rc, phi, st = m.read()
    lat = step_latency(torch, m, w.dt, opts, samples=min(100, max(10, args.steps)))
    buckets = []
    for b in range(nb):
        n, K_b, vt, sw = P.sl_bucket_stats(m.h, b)
        fl = advect2d_flops_per_element(n, 4, sw, vt) * K_b
        adv_us = avg_us(acc, P.KER_MIX_ADV + b)
        buckets.append({"n": n, "elements": K_b, "vel_terms": vt, "remap_sweeps_mean": sw,
                        "advect_us": adv_us, "constrain_us": avg_us(acc, P.KER_MIX_CON + b),
                        "advect_flops": fl, "advect_TFLOPs": fl / (adv_us * 1e-6) / 1e12})
    m.read()
    m.close()
    # stated error: round trip under the steady swirl
    rt = 100
    wr = W.c4(nsteps=rt)
    mr = P.from_mixed_workload(wr, stream=stream.cuda_stream, precision=prec)
    mr.step(wr.dt, rt, **opts)
    mr.set_velocity(-wr.velocity())
    mr.step(wr.dt, rt, **opts)
    rrc, back, _ = mr.read()
    mr.close()
    wr.exact = lambda x, y, t: wr.u0(x, y)
    l2 = wr.l2_error(back, 0.0)
    l2_ref = wr.l2_error(np.zeros_like(back), 0.0)

    # the dominant kernel: the longest launch of the step (the advect of the
    # highest-order bucket; its constrain launches are a fraction of it)
    dom = max(buckets, key=lambda d: d["advect_us"])
    assert dom["advect_us"] >= max(d["constrain_us"] for d in buckets)
    ach = dom["advect_flops"] / (dom["advect_us"] * 1e-6)
    counts = {int(n) - 1: int((w.orders == n).sum()) for n in sorted(set(w.orders.tolist()))}
    out = {
        "metric": METRIC, "value": w.dofs * args.steps / el, "unit": "DOF-updates/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": el / args.steps * 1e3, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f64", "data": "synthetic",
        "config": {"workload": "2D mixed-order batch: 316x316 quads on [0,1]^2, order per element from {4,6,8,12} "
                               "by seed, swirl a=(sin^2(pi x)sin(2pi y), -sin^2(pi y)sin(2pi x)), eight Fourier "
                               "modes, periodic, boundary HARD, RK4, graph-captured buckets, autotuned shapes",
                   "K": w.K, "dofs": w.dofs, "dt": w.dt, "elements_per_order": counts,
                   "precision": args.precision},
        "status": P.status_string(rc),
        "l2_error": l2, "l2_error_note": f"forward {rt} steps, velocity reversed, {rt} steps back; exact result "
                                         f"= u0 (paper's L2 norm, eq. 5.2; the norm of u0 itself is {l2_ref:.3g})",
        "round_trip_status": P.status_string(rrc),
        "step_latency": lat,
        "remap_sweeps_mean": st.remap_sweeps_mean,
        "eager_step_ms": avg_us(acc, P.KER_ADV2D) / 1e3,
        "graph_step_ms": el / args.steps * 1e3,
        "buckets": buckets,
        "roofline": {"kernel": f"k_advect2d (n={dom['n']} bucket)", "bound": "alu", "achieved": ach / 1e12,
                     "peak": FP64_VALU_PEAK / 1e12, "unit": "TFLOP/s", "frac": ach / FP64_VALU_PEAK,
                     "traffic": measured_traffic(f"k_advect2d_n{dom['n']}", "sl2d_kernels.h",
                                                 "sl2d_c4_mixed_316x316.md") if args.precision == "fp64" else None,
                     "avg_launch_us": dom["advect_us"], "algorithmic_flops_per_launch": dom["advect_flops"],
                     "elements_per_launch": dom["elements"], "remap_sweeps_mean": dom["remap_sweeps_mean"]},
    }
    if not args.no_cpu:
        out["cpu_baseline"] = cpu_baseline_mixed(W.c4(kx=16, nsteps=1))
    print(json.dumps(out))


def serve_stream(W, count, seed):
    """Seeded request mix of the serving configuration: dim 1 or 2 (p = 1/2);
    K uniform in [64, 65536] (2D: kx = ky = round(sqrt K)); order N uniform in
    {4..16}; 1D u0 the C2 Gaussian or a random sine field, 2D the C3 hill
    with its exact inflow; velocity of C2 (1D) or C3 (2D); 10..500 steps; 2D
    requests FP64 or FP32-refined (p = 1/2; order 16 runs in FP64 only).
    Inputs are built only when a request is submitted."""
    rng = np.random.default_rng(seed)
    specs = []
    for i in range(count):
        dim = int(rng.integers(1, 3))
        K = int(rng.integers(64, 65537))
        steps = int(rng.integers(10, 501))
        if dim == 1:
            N = int(rng.integers(4, 17))
            specs.append(dict(dim=1, K=K, n=N + 1, steps=steps, sine=bool(rng.integers(0, 2)), prec=0, seed=i))
        else:
            k = max(1, int(round(math.sqrt(K))))
            N = int(rng.integers(4, 17))
            prec = int(rng.integers(0, 2))
            specs.append(dict(dim=2, K=k * k, kx=k, n=N + 1, steps=steps, prec=prec if N < 16 else 0, seed=i))
    return specs


def serve_stream_small(W, count, seed):
    """Seeded stream of small requests, where requests of one kernel variant
    meet on the device: 1D (p = 1/2) with K uniform in [64, 1024] and N in
    {8, 16}, the C2 velocity and u0; 2D with kx = ky uniform in [4, 12] and
    N in {6, 8}, the C3 problem; FP64; 20..200 steps."""
    rng = np.random.default_rng(seed)
    specs = []
    for i in range(count):
        steps = int(rng.integers(20, 201))
        if int(rng.integers(1, 3)) == 1:
            K = int(rng.integers(64, 1025))
            specs.append(dict(dim=1, K=K, n=int(rng.choice([8, 16])) + 1, steps=steps, sine=False, prec=0, seed=i))
        else:
            k = int(rng.integers(4, 13))
            specs.append(dict(dim=2, K=k * k, kx=k, n=int(rng.choice([6, 8])) + 1, steps=steps, prec=0, seed=i))
    return specs


def serve_closed(P, W, specs, slots, budget, batch):
    """Capacity of the request loop on `specs` (all inputs built first, then
    submitted at once): DOF-updates/s, step latency, group-step sharing."""
    built = []
    for sp in specs:
        built.append(serve_inputs(W, sp))
    with P.Server(max_active=slots, hbm_budget=budget, batch=batch) as S:
        S.progress()
        t0 = time.perf_counter()
        ids, work = [], 0
        for args_, kw, wk in built:
            ids.append(S.submit(*args_, **kw))
            work += wk
        S.drain()
        wall = time.perf_counter() - t0
        p50, p99, samples, dof = S.latency()
        launches, member_steps = S.batching()
        for rid in ids:
            S.result(rid)
    return {"dof_per_s": dof / wall, "wall_s": wall, "step_p50_ms": p50, "step_p99_ms": p99,
            "request_steps_per_group_step": member_steps / launches if launches else None}


def serve_inputs(W, sp):
    """Positional and keyword arguments of Server.submit for one spec, and
    its DOF-updates."""
    if sp["dim"] == 1:
        w = W.c2(K=sp["K"], n=sp["n"], nsteps=sp["steps"], cmask=W.BOUNDARY)
        u0 = W.random_field_1d(w.K, w.n, sp["seed"], x0=w.x0, x1=w.x1) if sp["sine"] else w.initial()
        a, _ = w.velocity()
        ghost = None
    else:
        w = W.c3(kx=sp["kx"], n=sp["n"], nsteps=sp["steps"])
        u0 = w.initial()
        a, _ = w.velocity()
        ghost = w.ghost_rows(0.0, w.nsteps)
    kw = dict(dt=w.dt, nsteps=w.nsteps, ghost=ghost, nodes=w.family, bc=w.bc, form=w.form, precision=sp["prec"],
              x0=w.x0, x1=w.x1, y0=w.y0, y1=w.y1, rk=w.rk, constraints=w.cmask, mode=w.mode)
    return (w.dim, w.kx, w.ky, w.n - 1, u0, a), kw, w.K * w.nd * w.nsteps


def serve_submit(S, W, sp):
    pos, kw, wk = serve_inputs(W, sp)
    return S.submit(*pos, **kw), wk


def serve_pass(args, P, W, specs, batch):
    """One serving measurement of the request stream `specs`: a closed-loop
    pass (all submitted at once) for the capacity, then an open loop of
    seeded Poisson arrivals at 0.8x that capacity."""
    count = len(specs)
    budget = int(args.budget_gib * (1 << 30))
    with P.Server(max_active=args.slots, hbm_budget=budget, batch=batch) as S:
        t0 = time.perf_counter()
        ids, work = [], 0
        S.progress()
        for sp in specs:
            rid, wk = serve_submit(S, W, sp)
            ids.append(rid)
            work += wk
        S.drain()
        closed = time.perf_counter() - t0
        for rid in ids:
            S.result(rid)
    capacity = work / closed
    rng = np.random.default_rng(7)
    rate = 0.8 * capacity / (work / count)          # requests per second
    arrivals = np.cumsum(rng.exponential(1.0 / rate, size=count))
    statuses = []
    with P.Server(max_active=args.slots, hbm_budget=budget, batch=batch) as S:
        S.progress()  # the server's loop runs on its own threads from here
        t0 = time.perf_counter()
        ids, i = [], 0
        while i < count:
            now = time.perf_counter() - t0
            while i < count and arrivals[i] <= now:
                ids.append(serve_submit(S, W, specs[i])[0])
                i += 1
            if i < count:
                time.sleep(max(0.0, arrivals[i] - (time.perf_counter() - t0)))
        S.drain()
        wall = time.perf_counter() - t0
        p50, p99, samples, dof = S.latency()
        launches, member_steps = S.batching()
        lat_req = []
        for rid in ids:
            rc, _, _, tm = S.result(rid)
            statuses.append(rc)
            lat_req.append(tm.total_us)
    lat_req.sort()
    return {"value": dof / wall, "closed_loop_dof_per_s": capacity, "arrival_rate_per_s": rate,
            "step_latency": {"p50_ms": p50, "p99_ms": p99, "samples": samples},
            "request_latency_ms": {"p50": lat_req[len(lat_req) // 2] / 1e3,
                                   "p99": lat_req[min(len(lat_req) - 1, int(0.99 * len(lat_req)))] / 1e3},
            "failed_requests": int(sum(1 for r in statuses if r not in (P.SL_OK,))), "wall_s": wall,
            "group_steps": launches, "request_steps_per_group_step": member_steps / launches if launches else None}


def bench_serve(args, torch, P, W):
    """Serving: a seeded Poisson stream of independent problems through the
    request loop (continuous batching).  Small requests of one kernel
    variant are stepped together, one launch of each step kernel per group
    step; the same stream with every request on its own stream is measured
    beside it.  value = DOF-updates/s of the batched open loop, with the
    per-step latency p50/p99 of its requests.  A stream of small requests,
    where batching carries several requests per launch, is measured both
    ways as well (closed loop)."""
    specs = serve_stream(W, args.requests, seed=2024)
    # untimed pass first: the first launch of each kernel loads its code and
    # the clocks rise from idle, a cost the first measured pass would carry
    serve_closed(P, W, specs, args.slots, int(args.budget_gib * (1 << 30)), True)
    b = serve_pass(args, P, W, specs, True)
    u = serve_pass(args, P, W, specs, False)
    small = serve_stream_small(W, 256, seed=77)
    budget = int(args.budget_gib * (1 << 30))
    serve_closed(P, W, small, 32, budget, True)  # untimed, as above
    sb = serve_closed(P, W, small, 32, budget, True)
    su = serve_closed(P, W, small, 32, budget, False)
    out = {
        "metric": METRIC, "value": b["value"], "unit": "DOF-updates/s", "n_gpus": 1,
        "steps": int(b["step_latency"]["samples"]), "warmup": 0, "ms_per_step": None, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f64 (2D requests half FP32-refined)", "data": "synthetic",
        "config": {"workload": f"serving: {args.requests} seeded Poisson arrivals of 1D (C2 velocity) and 2D (C3 "
                               "rotation) problems, K in [64,65536], N in 4..16, 10-500 steps, boundary rows",
                   "slots": args.slots, "hbm_budget_gib": args.budget_gib,
                   "arrival_rate_per_s": b["arrival_rate_per_s"],
                   "closed_loop_dof_per_s": b["closed_loop_dof_per_s"]},
        "step_latency": b["step_latency"], "request_latency_ms": b["request_latency_ms"],
        "failed_requests": b["failed_requests"], "wall_s": b["wall_s"],
        "batching": {"group_steps": b["group_steps"],
                     "request_steps_per_group_step": b["request_steps_per_group_step"]},
        "unbatched": {k: u[k] for k in ("value", "closed_loop_dof_per_s", "step_latency", "request_latency_ms",
                                        "failed_requests", "wall_s")},
        "small_requests": {"workload": "256 small requests (1D K in [64,1024], N in {8,16}; 2D 4x4..12x12, N in "
                                       "{6,8}; FP64; 20-200 steps), all submitted at once, 32 slots",
                           "batched": sb, "unbatched": su},
    }
    print(json.dumps(out))


def bench_c1(args, torch, P, W, stream):
    """The small 1D configuration: u_t + u_x = 0 on [0,2] periodic, K=16,
    order 8 (144 DOF), RK4, boundary rows, dt = 1.6516e-3.  Far too small to
    load the GPU: what it measures is the cost of a step's launches, as a
    stream of steps (one sl_step of `steps` steps) and as the served latency
    of single steps.  No roofline claim is made for it."""
    w = W.c1()
    m = P.from_workload(w, stream=stream.cuda_stream)
    opts = dict(rk=w.rk, constraints=w.cmask, mode=w.mode)
    m.step(w.dt, args.warmup, **opts)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    m.step(w.dt, args.steps, **opts)
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    rc, phi, st = m.read()
    T = (args.warmup + args.steps) * w.dt
    l2 = w.l2_error(phi, T)
    lat = step_latency(torch, m, w.dt, opts, samples=min(200, max(10, args.steps)))
    P.sl_set_profiling(m.h, True)
    m.step(w.dt, 50, **opts)
    t_adv, c_adv = P.sl_kernel_time(m.h, P.KER_ADV1D)
    t_con, c_con = P.sl_kernel_time(m.h, P.KER_CON1D)
    P.sl_set_profiling(m.h, False)
    m.close()
    out = {
        "metric": METRIC, "value": w.dofs * args.steps / el, "unit": "DOF-updates/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": el / args.steps * 1e3, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f64", "data": "synthetic",
        "config": {"workload": "1D u_t+u_x=0 on [0,2] periodic, K=16, order 8 (9 GL nodes), u0=sin(pi x), RK4, "
                               "boundary HARD, dt=0.2*gap*dx", "K": w.K, "n": w.n, "dofs": w.dofs, "dt": w.dt},
        "l2_error": l2, "l2_time": T, "status": P.status_string(rc),
        "step_latency": lat,
        "kernels_us": {"sl1d_advect": t_adv / max(c_adv, 1) * 1e3, "sl1d_constrain": t_con / max(c_con, 1) * 1e3},
        "roofline": None,
    }
    print(json.dumps(out))


def bench_c2bw(args, torch, P, W, stream):
    """The HBM side of the 1D step: the C2 problem (order 16, RK4, the same
    velocity and initial data) with boundary rows only, on K = 2^22 elements
    (71.3 M DOF, 0.57 GB per nodal array), far beyond the last-level cache.
    Without targets the advect kernel carries about 2.7 kflop per element
    against about 0.46 kB, so both kernels are bound by HBM."""
    w = W.c2(K=1 << 22, cmask=W.BOUNDARY)
    steps = max(1, min(args.steps, 200))
    warm = max(1, min(args.warmup, 20))
    m = P.from_workload(w, stream=stream.cuda_stream)
    opts = dict(rk=w.rk, constraints=w.cmask, mode=w.mode)
    m.step(w.dt, warm, **opts)
    kinds = [P.KER_ADV1D, P.KER_CON1D]
    acc = profiled_window(P, m, w.dt, 10, opts, kinds)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    m.step(w.dt, steps, **opts)
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    profiled_window(P, m, w.dt, 10, opts, kinds, acc)
    rc, phi, st = m.read()
    T = st.t
    l2 = w.l2_error(phi, T)
    m.close()

    adv_avg = avg_us(acc, P.KER_ADV1D) * 1e-6
    con_avg = avg_us(acc, P.KER_CON1D) * 1e-6
    by_a = advect_bytes_per_element(w.n, False, st.vel_terms) * w.K
    by_c = constrain_bytes_per_element(w.n, False) * w.K
    fl_a = advect_flops_per_element(w.n, 4, 3, False, st.vel_terms) * w.K
    kern = {"sl1d_advect": {"avg_launch_us": adv_avg * 1e6, "algorithmic_bytes_per_launch": by_a,
                            "achieved_GBps": by_a / adv_avg / 1e9, "frac_hbm": by_a / adv_avg / HBM_PEAK,
                            "algorithmic_flops_per_launch": fl_a,
                            "achieved_TFLOPs": fl_a / adv_avg / 1e12},
            "sl1d_constrain": {"avg_launch_us": con_avg * 1e6, "algorithmic_bytes_per_launch": by_c,
                               "achieved_GBps": by_c / con_avg / 1e9, "frac_hbm": by_c / con_avg / HBM_PEAK}}
    dom, by, avg = ("sl1d_advect", by_a, adv_avg) if adv_avg >= con_avg else ("sl1d_constrain", by_c, con_avg)
    roof = {"kernel": dom, "bound": "hbm", "achieved": by / avg / 1e9, "peak": HBM_PEAK / 1e9, "unit": "GB/s",
            "frac": by / avg / HBM_PEAK,
            "traffic": measured_traffic("k_advect1d" if dom == "sl1d_advect" else "k_constrain1d",
                                        profile="sl1d_c2bw_K4194304_n17.md"),
            "avg_launch_us": avg * 1e6, "algorithmic_bytes_per_launch": by, "kernels": kern}
    out = {
        "metric": METRIC, "value": w.dofs * steps / el, "unit": "DOF-updates/s", "n_gpus": 1, "steps": steps,
        "warmup": warm, "ms_per_step": el / steps * 1e3, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f64", "data": "synthetic",
        "config": {"workload": "HBM probe: 1D a(x)=1+0.5sin(pi x) on [0,2] periodic, K=2^22, order 16 (17 GL "
                               "nodes), u0=exp(-40(x-1)^2), RK4, boundary rows only, HARD, dt=0.2*gap*dx/1.5",
                   "K": w.K, "n": w.n, "dofs": w.dofs, "dt": w.dt, "rk": w.rk, "constraints": "B"},
        "l2_error": l2, "l2_time": T, "status": P.status_string(rc),
        "roofline": roof,
    }
    if not args.no_cpu:
        piece = W.c2(cmask=W.BOUNDARY)
        cb = cpu_baseline(piece)
        cb["sample"] = "a K=65536 piece of the same problem (the same work per element): " + cb["sample"]
        out["cpu_baseline"] = cb
    print(json.dumps(out))


def bench_c2(args, torch, P, W, stream):
    """1D variable-velocity advection a(x) = 1 + sin(pi x)/2 on [0,2]
    periodic, K = 65536 elements of order 16 (17 Gauss-Legendre nodes,
    1,114,112 DOF), u0 = exp(-40 (x-1)^2), RK4, boundary + mass + energy
    constraints (HARD, the paper's energy stop 1e-8), dt = 0.2 * min node gap
    * dx / 1.5, FP64."""
    w = W.c2()
    m = P.from_workload(w, stream=stream.cuda_stream)
    opts = dict(rk=w.rk, constraints=w.cmask, mode=w.mode, energy_maxit=w.energy_maxit, energy_tol=w.energy_tol)

    m.step(w.dt, args.warmup, **opts)
    kinds = [P.KER_ADV1D, P.KER_CON1D]
    nprof = max(10, min(args.steps, 200))
    acc = profiled_window(P, m, w.dt, nprof, opts, kinds)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    m.step(w.dt, args.steps, **opts)
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    profiled_window(P, m, w.dt, nprof, opts, kinds, acc)
    rc, phi, st = m.read()
    T = st.t
    l2 = w.l2_error(phi, T)
    lat = step_latency(torch, m, w.dt, opts, samples=min(200, max(10, args.steps)))
    m.read()
    m.close()
    t_adv, c_adv = acc[P.KER_ADV1D]
    t_con, c_con = acc[P.KER_CON1D]

    s_stages = 4
    nq = 3
    targets = True
    fl = advect_flops_per_element(w.n, s_stages, nq, targets, st.vel_terms) * w.K
    by = advect_bytes_per_element(w.n, targets, st.vel_terms) * w.K
    adv_avg = t_adv / max(c_adv, 1) * 1e-3
    con_avg = t_con / max(c_con, 1) * 1e-3
    if adv_avg >= con_avg:
        ach = fl / adv_avg
        roof = {"kernel": "sl1d_advect", "bound": "alu", "achieved": ach / 1e12, "peak": FP64_VALU_PEAK / 1e12,
                "unit": "TFLOP/s", "frac": ach / FP64_VALU_PEAK, "traffic": measured_traffic("k_advect1d"),
                "avg_launch_us": adv_avg * 1e6, "algorithmic_flops_per_launch": fl,
                "algorithmic_bytes_per_launch": by, "velocity_series_terms": st.vel_terms}
    else:
        cb = constrain_bytes_per_element(w.n) * w.K
        ach = cb / con_avg
        roof = {"kernel": "sl1d_constrain", "bound": "hbm", "achieved": ach / 1e9, "peak": HBM_PEAK / 1e9,
                "unit": "GB/s", "frac": ach / HBM_PEAK, "traffic": measured_traffic("k_constrain1d"),
                "avg_launch_us": con_avg * 1e6,
                "algorithmic_bytes_per_launch": cb}
    roof["kernels_us"] = {"sl1d_advect": adv_avg * 1e6, "sl1d_constrain": con_avg * 1e6}

    value = w.dofs * args.steps / el
    out = {
        "metric": METRIC, "value": value, "unit": "DOF-updates/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": el / args.steps * 1e3, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f64", "data": "synthetic",
        "config": {"workload": "1D a(x)=1+0.5sin(pi x) on [0,2] periodic, K=65536, order 16 (17 GL nodes), "
                               "u0=exp(-40(x-1)^2), RK4, boundary+mass+energy HARD, dt=0.2*gap*dx/1.5",
                   "K": w.K, "n": w.n, "dofs": w.dofs, "dt": w.dt, "rk": w.rk, "constraints": "B+M+E",
                   "energy_tol": w.energy_tol},
        "l2_error": l2, "l2_time": T, "status": P.status_string(rc), "max_picard": st.max_picard,
        "step_latency": lat,
        "roofline": roof,
    }
    if not args.no_cpu:
        out["cpu_baseline"] = cpu_baseline(w)
    print(json.dumps(out))



def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=1000)
    ap.add_argument("--warmup", type=int, default=50)
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--workload", choices=["c1", "c2", "c2bw", "c3", "c4", "serve"], default="c4",
                    help="c4: the 2D mixed-order batch, the largest configuration (default); "
                         "c1: the small 1D configuration (144 DOF), a launch-latency probe; "
                         "c2: the 1D configuration with boundary, mass and energy rows; c2bw: the C2 problem "
                         "with boundary rows only on K=2^22 elements, a probe of the HBM side; "
                         "c3: the 2D rotation configuration; "
                         "serve: a Poisson stream of independent problems through the request loop")
    ap.add_argument("--requests", type=int, default=48, help="serve: number of requests")
    ap.add_argument("--slots", type=int, default=8, help="serve: requests on the device at once")
    ap.add_argument("--budget-gib", type=float, default=32.0, help="serve: device memory budget")
    ap.add_argument("--constraints", choices=["b", "bm", "bme"], default="b",
                    help="c3: boundary rows (default), + mass, + mass and energy (HARD)")
    ap.add_argument("--precision", choices=["fp64", "fp32r", "bf16r"], default="fp64",
                    help="c3 and c4: fp32r stores and applies the remap preconditioner in FP32, bf16r with BF16 "
                         "entries and operands and FP32 sums (FP64 residuals in both)")
    ap.add_argument("--copy-mib", type=int, default=0,
                    help="first run one plain device copy of this many MiB (calibrates HBM counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only (asked for --gpus {args.gpus}); "
              "the multi-GPU path is a design note, not a build target.", file=sys.stderr)
        sys.exit(2)

    import torch
    import paper_1910_06476_amd as P
    import workloads as W

    if not torch.cuda.is_available():
        print("no GPU visible", file=sys.stderr)
        sys.exit(1)
    torch.cuda.set_device(0)
    stream = torch.cuda.current_stream()
    if args.copy_mib > 0:
        nel = args.copy_mib * (1 << 20) // 8
        src = torch.ones(nel, dtype=torch.float64, device="cuda")
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    if args.workload == "c3":
        return bench_c3(args, torch, P, W, stream)
    if args.workload == "serve":
        return bench_serve(args, torch, P, W)
    if args.workload == "c4":
        return bench_c4(args, torch, P, W, stream)
    if args.workload == "c2bw":
        return bench_c2bw(args, torch, P, W, stream)
    if args.workload == "c1":
        return bench_c1(args, torch, P, W, stream)
    return bench_c2(args, torch, P, W, stream)

if __name__ == "__main__":
    main()
