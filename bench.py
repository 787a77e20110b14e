"""Benchmark of the explicit semi-Lagrangian spectral step on one MI355X.

Workload (the headline configuration): 1D variable-velocity advection
a(x) = 1 + sin(pi x)/2 on [0,2] periodic, K = 65536 elements of order 16
(17 Gauss-Legendre nodes, 1,114,112 DOF), u0 = exp(-40 (x-1)^2), RK4,
boundary + mass + energy constraints (HARD), dt = 0.2 * min node gap * dx /
1.5, FP64.  One "step" is one sl_step over the whole mesh (all stages of the
method).  Inputs are resident in HBM before the timed region.

Prints one JSON line: DOF-updates/s over K timed steps, the L2 error against
the closed-form solution at the final time, the roofline of the dominant
kernel (HIP events on the mesh's stream, algorithmic flop count per element
as stated in the design doc), and the CPU oracle timed on a bounded sample.
"""
from __future__ import annotations

import argparse
import json
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
    Clenshaw evaluation 3 flops per term (vel_terms terms for the velocity
    series, n for phi^n); RK stage update ~4 flops per stage."""
    clen = 3.0 * n
    clen_v = 3.0 * vel_terms
    rk_move = (s - 1) * clen_v + 4.0 * s
    f = n * rk_move                      # forward motion of the n particles
    f += n * (2.0 * n)                   # moved-point weights lambda*: n-1 (sub, mul) + div
    f += n * (5.0 * n) + 2 * 5.0 * n     # remap at n nodes + 2 edge traces (product form)
    if targets:
        f += 2.0 * n * n                 # Chebyshev coefficients of phi^n
        back = rk_move + clen            # one backtrace + evaluation of phi^n at its foot
        f += n * (nq - 1) * (back + 6)   # node backtraces (volume term)
        f += 2 * ((nq - 1) * (back + 4) + clen)  # edge values at the RK abscissae
        f += 8.0 * n                     # mass/energy sums
    return f


def advect_bytes_per_element(n: int, targets: bool) -> float:
    """Algorithmic HBM bytes of the 1D advect kernel per element: read phi,
    nodal and modal velocity (+ nodal divergence with targets), write phihat
    and the 8-double element record."""
    return 8.0 * n * (3 + (1 if targets else 0)) + 8.0 * n + 64.0


def constrain_bytes_per_element(n: int) -> float:
    """read phihat, the element record (neighbours' are cache hits), two face
    velocities; write phi."""
    return 8.0 * n + 64.0 + 8.0 + 8.0 * n


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


def cpu_baseline(w, budget_s: float = 12.0):
    import oracle
    oracle.build(force=False)
    p = oracle.params_from(w)
    a, _ = w.velocity()
    phi = w.initial()
    t0 = time.perf_counter()
    phi, _ = oracle.step(p, phi, a=a, dt=w.dt, nsteps=1)
    one = time.perf_counter() - t0
    steps = max(1, min(50, int(budget_s / max(one, 1e-3))))
    t0 = time.perf_counter()
    oracle.step(p, phi, a=a, dt=w.dt, nsteps=steps)
    el = time.perf_counter() - t0
    cores = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    return {"value": w.dofs * steps / el, "unit": "DOF-updates/s", "cores": cores, "kind": "oracle",
            "sample": f"full mesh (K={w.K}, n={w.n}), {steps} steps after 1 warm-up step, "
                      f"{el:.1f} s, OpenMP threads={cores}"}


def advect2d_flops_per_element(n: int, s: int, sweeps: float, vel_terms: int) -> float:
    """Algorithmic FP64 flops of the 2D advect+solve kernel per element:
    motion (tensor Clenshaw, 2 components, (s-1) evaluations per particle,
    3 flops per term), the V rows (product form, ~6n per particle), the
    separable preconditioner (2 n^2 (n-1) products to build, 4 n^3 per
    application), and per defect-correction sweep the matrix-free V x
    (2 n^4 + 2 n^2) plus one preconditioner application."""
    nd = n * n
    m = vel_terms
    clen2 = 3.0 * (m * m + m)
    f = nd * ((s - 1) * 2 * clen2 + 8.0 * s)
    f += nd * 6.0 * n
    f += 2 * nd * 4.0 * (n - 1)
    apply = 4.0 * n ** 3
    f += apply
    f += sweeps * (2.0 * n ** 4 + 2.0 * nd + apply + 2.0 * nd)
    f += 4 * n * 2.0 * n
    return f


def bench_c3(args, torch, P, W, stream):
    """2D rotation workload (256x256, order 8, RK4, ghost inflow, boundary HARD)."""
    w = W.c3(nsteps=args.warmup + args.steps)
    prec = P.SL_PREC_FP32_REFINED if args.precision == "fp32r" else P.SL_PREC_FP64
    m = P.from_workload(w, stream=stream.cuda_stream, precision=prec)
    m.set_ghost(w.ghost_rows(0.0, args.warmup + 2 * args.steps + 20))
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
    sweeps = st.remap_sweeps_mean  # defect-correction sweeps per element and step, measured
    nprof = max(5, min(args.steps, 20))
    P.sl_set_profiling(m.h, True)
    m.step(w.dt, nprof, **opts)
    t_adv, c_adv = P.sl_kernel_time(m.h, P.KER_ADV2D)
    t_con, c_con = P.sl_kernel_time(m.h, P.KER_CON2D)
    P.sl_set_profiling(m.h, False)
    m.close()
    adv_avg = t_adv / max(c_adv, 1) * 1e-3
    con_avg = t_con / max(c_con, 1) * 1e-3
    fl = advect2d_flops_per_element(w.n, 4, sweeps, st.vel_terms) * w.K
    ach = fl / adv_avg
    out = {
        "metric": METRIC, "value": w.dofs * args.steps / el, "unit": "DOF-updates/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": el / args.steps * 1e3,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f64", "data": "synthetic",
        "config": {"workload": "2D rotation a=(-(y-1/2),x-1/2) on [0,1]^2, 256x256, order 8 (81 nodes/elem), "
                               "Gaussian hill, RK4, ghost inflow from the exact solution, boundary HARD",
                   "K": w.K, "n": w.n, "dofs": w.dofs, "dt": w.dt},
        "l2_error": l2, "l2_time": T, "status": P.status_string(rc), "precision": args.precision,
        "remap_sweeps_mean": sweeps, "remap_sweeps_max": st.remap_sweeps_max, "refine_resid": st.refine_resid,
        "vel_terms": st.vel_terms,
        "roofline": {"kernel": "sl2d_advect", "bound": "alu", "achieved": ach / 1e12,
                     "peak": FP64_VALU_PEAK / 1e12, "unit": "TFLOP/s", "frac": ach / FP64_VALU_PEAK,
                     "traffic": measured_traffic("k_advect2d", "sl2d.hip", "sl2d_c3_256x256_n9.md")
                     if args.precision == "fp64" else None,
                     "avg_launch_us": adv_avg * 1e6, "algorithmic_flops_per_launch": fl,
                     "kernels_us": {"sl2d_advect": adv_avg * 1e6, "sl2d_constrain": con_avg * 1e6}},
    }
    print(json.dumps(out))


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=1000)
    ap.add_argument("--warmup", type=int, default=50)
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--workload", choices=["c2", "c3"], default="c2",
                    help="c2: the headline 1D configuration (default); c3: the 2D rotation configuration")
    ap.add_argument("--precision", choices=["fp64", "fp32r"], default="fp64",
                    help="c3 only: fp32r stores and applies the remap preconditioner in FP32 (FP64 residuals)")
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
    w = W.c2()
    m = P.from_workload(w, stream=stream.cuda_stream)
    opts = dict(rk=w.rk, constraints=w.cmask, mode=w.mode, energy_maxit=w.energy_maxit, energy_tol=w.energy_tol)

    m.step(w.dt, args.warmup, **opts)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    m.step(w.dt, args.steps, **opts)
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    rc, phi, st = m.read()
    T = (args.warmup + args.steps) * w.dt
    l2 = w.l2_error(phi, T)

    # per-kernel HIP-event timing on the mesh's stream (a second pass)
    nprof = max(10, min(args.steps, 200))
    P.sl_set_profiling(m.h, True)
    m.step(w.dt, nprof, **opts)
    t_adv, c_adv = P.sl_kernel_time(m.h, P.KER_ADV1D)
    t_con, c_con = P.sl_kernel_time(m.h, P.KER_CON1D)
    P.sl_set_profiling(m.h, False)
    m.read()
    m.close()

    s_stages = 4
    nq = 3
    targets = True
    fl = advect_flops_per_element(w.n, s_stages, nq, targets, st.vel_terms) * w.K
    by = advect_bytes_per_element(w.n, targets) * w.K
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
        "roofline": roof,
    }
    if not args.no_cpu:
        out["cpu_baseline"] = cpu_baseline(w)
    print(json.dumps(out))


if __name__ == "__main__":
    main()
