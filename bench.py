#!/usr/bin/env python
"""Benchmark of the partitioned shift-without-invert eigensolve + T(E).

One step = the whole hot path on one synthetic system: operator build,
window planning (Algorithm 1: E_min/E_max from two exterior solves, then the
shifts), the batched solve of every window to backward error 1e-8, the
combine (Algorithm 2) and T(E) at the workload's energies.  Inputs are made
on the host once; the timed region starts with the device idle.

Metric: converged (unique, after combine) eigenpairs per second.
Prints ONE JSON line.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0


def energy_grid(eps, n):
    import numpy as np
    re = np.asarray(eps).real
    return np.linspace(re.min(), re.max(), n) if n > 1 else np.array([re.mean()])


def run_step(w, prec_code, n_r, p, opts, max_windows=None, plan="semiclassical"):
    from paper_1606_01139_amd import Operator, PLAN_EQUAL, PLAN_SAMPLED, PLAN_SEMICLASSICAL
    g = w.grid
    oper = Operator(g.nx, g.ny, g.nz, g.h, w.V, w.absorber.as_tuple())
    t0 = time.perf_counter()
    mode = {"semiclassical": PLAN_SEMICLASSICAL, "sampled": PLAN_SAMPLED, "alg1": PLAN_EQUAL}[plan]
    wins, erange = oper.plan_windows(n_r, p, mode, opts)
    oper.plan_seconds = time.perf_counter() - t0
    if max_windows:
        wins = wins[:max_windows]
    n, holes, status = oper.solve_all_partitions(wins, opts, allow_noconv=True)
    eps = oper.eigenvalues()
    T = oper.transmission(energy_grid(eps, w.n_energies)) if w.n_energies else None
    stats = [oper.stats(j) for j in range(len(wins))]
    return oper, n, holes, status, wins, erange, stats, T


def stencil_roofline(w, ncols, dtype, reps=50):
    """Average duration of the stencil kernel in the solver's launch shape
    (one block of ncols vectors), timed with HIP events on the stream the
    library launches on."""
    import numpy as np
    import torch
    from paper_1606_01139_amd import Operator
    g = w.grid
    oper = Operator(g.nx, g.ny, g.nz, g.h, w.V, w.absorber.as_tuple())
    N = g.n
    tdt = torch.complex128 if dtype == "c128" else torch.complex64
    X = torch.randn(ncols, N, dtype=tdt, device="cuda")
    Y = torch.empty_like(X)
    for _ in range(5):
        oper.apply(X, Y)
    torch.cuda.synchronize()
    st = torch.cuda.current_stream()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(st)
    for _ in range(reps):
        oper.apply(X, Y)
    e1.record(st)
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / reps
    s_c = 16 if dtype == "c128" else 8
    s_r = 8 if dtype == "c128" else 4
    bytes_alg = 2 * N * ncols * s_c + N * s_r + g.nz * s_r
    gbs = bytes_alg / (ms * 1e-3) / 1e9
    oper.close()
    return {"bound": "hbm", "achieved": round(gbs, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": round(gbs / HBM_PEAK_GBS, 4), "traffic": None,
            "kernel": f"stencil_kernel<{'double' if dtype == 'c128' else 'float'},6>",
            "launch": f"N={N} x {ncols} cols", "avg_ms": round(ms, 5), "algorithmic_bytes": bytes_alg}


def cpu_baseline(w, seconds_cap=30.0):
    """The oracle (ARPACK 'SM' on the shifted operator, FP64, CPU) on a bounded
    sample of the same workload: the window nearest the bottom of the
    spectrum with a reduced count, timed on the host cores."""
    import numpy as np
    from oracle import operator as op, eigen
    g = w.grid
    ab = w.absorber.as_tuple()
    gL, gR = op.gamma_fields(g.nx, g.ny, g.nz, g.h, ab)
    A = op.assemble_sparse(g.nx, g.ny, g.nz, g.h, w.V, gL, gR)
    t0 = time.perf_counter()
    emin = eigen.extremal_real(A, "SR", False).real
    nev = 10
    e, U = eigen.window_arpack(A, emin + 0.3, nev)
    dt = time.perf_counter() - t0
    cores = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    return {"value": round(nev / dt, 4), "unit": "eigenpairs/s", "cores": cores, "kind": "oracle",
            "sample": f"one window of {nev} eigenpairs nearest E_min+0.3 Ha (plus the E_min solve) on the "
                      f"{g.nx}x{g.ny}x{g.nz} grid, ARPACK SM on the shifted operator, {dt:.1f} s"}


def main():
    ap = argparse.ArgumentParser(description=__doc__)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=2)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--config", default="c2")
    ap.add_argument("--precision", default="bulk", choices=["fp64", "bulk"])
    ap.add_argument("--max-restarts", type=int, default=2000)
    ap.add_argument("--max-windows", type=int, default=0)
    ap.add_argument("--plan", default="semiclassical", choices=["semiclassical", "sampled", "alg1"])
    ap.add_argument("--block", type=int, default=0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--verbose", action="store_true")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {args.gpus}); "
              "the windows would be dealt across GPUs as described in DESIGN.md", file=sys.stderr)
        sys.exit(2)
    import numpy as np
    import torch
    from paper_1606_01139_amd import default_opts, FP64, FP32_BULK
    from synth.workloads import workload

    torch.cuda.set_device(0)
    w = workload(args.config)
    p, nev = w.n_windows, w.nev_per_window
    n_r = p * nev
    prec = FP64 if args.precision == "fp64" else FP32_BULK
    opts = default_opts(precision=prec, tol=1e-8, max_restarts=args.max_restarts)
    if args.block:
        opts.block = args.block
    for i in range(args.warmup):
        t = time.perf_counter()
        r = run_step(w, prec, n_r, p, opts, args.max_windows or None, args.plan)
        torch.cuda.synchronize()
        if args.verbose:
            print(f"warmup {i}: {time.perf_counter() - t:.2f} s, n={r[1]}", file=sys.stderr, flush=True)
        r[0].close()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    total = 0
    last = None
    for i in range(args.steps):
        r = run_step(w, prec, n_r, p, opts, args.max_windows or None, args.plan)
        total += r[1]
        if last is not None:
            last[0].close()
        last = r
        if args.verbose:
            print(f"step {i}: {time.perf_counter() - t0:.2f} s cumulative, n={r[1]}", file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    oper, n, holes, status, wins, erange, stats, T = last
    ms = dt / args.steps * 1e3
    b = opts.block
    roof = stencil_roofline(w, b * len(wins), "c64" if prec == FP32_BULK else "c128")
    out = {
        "metric": "converged eigenpairs/s at rel. residual 1e-8",
        "value": round(total / dt, 3),
        "unit": "eigenpairs/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms, 2),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "c64+f64" if prec == FP32_BULK else "f64",
        "data": "synthetic",
        "config": {"workload": f"{args.config}: {w.grid.nx}x{w.grid.ny}x{w.grid.nz} grid (N={w.grid.n}), "
                               f"{len(w.wells)} Gaussian wells, {len(wins)} windows x {nev} eigenpairs, "
                               f"T(E) at {w.n_energies} energies",
                   "precision": args.precision, "unique_eigenpairs": n, "holes": holes,
                   "status": int(status), "e_range": [round(x, 6) for x in erange],
                   "planner": args.plan, "plan_seconds_last_step": round(oper.plan_seconds, 3),
                   "block": opts.block},
        "roofline": roof,
        "windows": [{"shift": round(s.shift, 6), "nev": s.nev, "n_conv": s.n_conv, "restarts": s.restarts,
                     "restarts_bulk": s.restarts_bulk, "matvecs": s.matvecs,
                     "max_backward_error": s.max_backward_error} for s in stats],
    }
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(w)
    print(json.dumps(out), flush=True)
    oper.close()


if __name__ == "__main__":
    main()
