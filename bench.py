#!/usr/bin/env python
"""Benchmark of the partitioned shift-without-invert eigensolve + T(E).

One step = the whole hot path on one synthetic system: operator build,
window planning (E_min by an exterior solve, shifts from the counting
function), the batched solve of every window to backward error 1e-8, the
combine (Algorithm 2) and T(E) at the workload's energies.  Inputs are made
on the host once; the timed region starts with the device idle.

Metric: converged (unique, after combine) eigenpairs per second.
Prints ONE JSON line; progress goes to stderr.
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
FP64_PEAK_TFLOPS = 78.6


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def energy_grid(eps, n):
    import numpy as np
    re = np.asarray(eps).real
    return np.linspace(re.min(), re.max(), n) if n > 1 else np.array([re.mean()])


def run_step(w, n_r, p, opts, max_windows=None, plan="semiclassical", fill_rounds=0):
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
    oper.fill = {"rounds": 0, "inserted": 0, "holes_left": int(sum(holes))}
    if fill_rounds:
        # Algorithm 1's repeat loop: partitions inserted where no redundancy
        # was found, and above E_min if the first window does not reach it
        added, rounds, n, left, st2 = oper.fill_holes(erange[0], max(k for _, k in wins), fill_rounds, opts,
                                                      allow_noconv=True)
        oper.fill = {"rounds": rounds, "inserted": added, "holes_left": left}
        status = max(status, st2)
    eps = oper.eigenvalues()
    T = oper.transmission(energy_grid(eps, w.n_energies)) if w.n_energies else None
    stats = [oper.stats(j) for j in range(len(wins) + oper.fill["inserted"])]
    # a partition keeps only its pairs at backward error <= tol, so the
    # combined count is the converged count
    return oper, n, holes, status, wins, erange, stats, T


def run_batch(args):
    """Ragged batch (config c3): every window of every system in one batched
    iteration (tsg_solve_batch), complex64 bulk with FP64 small eigensolves
    and FP64 finish.  Planning (one exterior solve per system) is timed
    apart from the batched solve."""
    import torch
    from paper_1606_01139_amd import Operator, PLAN_SEMICLASSICAL, default_opts, solve_batch, FP32_BULK, FP64
    from synth.workloads import batch_workloads
    ws = batch_workloads(args.n_sys)
    prec = FP64 if args.precision == "fp64" else FP32_BULK
    opts = default_opts(precision=prec, tol=1e-8, max_restarts=args.max_restarts)
    if args.groups:
        opts.groups = args.groups
    t0 = time.perf_counter()
    ops, wins = [], []
    for w in ws:
        g = w.grid
        op = Operator(g.nx, g.ny, g.nz, g.h, w.V, w.absorber.as_tuple())
        wj, _ = op.plan_windows(w.n_windows * w.nev_per_window, w.n_windows, PLAN_SEMICLASSICAL, opts)
        ops.append(op)
        wins.append(wj)
    t_plan = time.perf_counter() - t0
    log(f"c3 planned {len(ws)} systems in {t_plan:.1f} s")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    nu, status = solve_batch(ops, wins, opts, allow_noconv=True)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    n_ok = 0
    worst = 0.0
    restarts = []
    for op, wj, n in zip(ops, wins, nu):
        st = [op.stats(j) for j in range(len(wj))]
        n_ok += n  # combined pairs are all at backward error <= tol
        worst = max([worst] + [s.max_backward_error for s in st if s.n_conv == s.nev])
        restarts += [s.restarts + s.restarts_bulk for s in st]
        op.close()
    Ns = [w.grid.n for w in ws]
    out = {"metric": "converged eigenpairs/s at rel. residual 1e-8", "value": round(n_ok / dt, 3),
           "unit": "eigenpairs/s", "n_gpus": 1, "steps": 1, "warmup": 0, "ms_per_step": round(dt * 1e3, 2),
           "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
           "dtype": "f64" if prec == FP64 else "c64+f64", "data": "synthetic",
           "config": {"workload": f"c3: {len(ws)} systems, N from {min(Ns)} to {max(Ns)} (total {sum(Ns)}), "
                                  f"{ws[0].n_windows} windows x {ws[0].nev_per_window} eigenpairs each, "
                                  "one batched iteration", "precision": args.precision,
                      "unique_converged_eigenpairs": n_ok, "status": int(status),
                      "plan_seconds": round(t_plan, 2), "max_backward_error": worst,
                      "restarts_max": max(restarts), "restarts_mean": round(sum(restarts) / len(restarts), 1)}}
    print(json.dumps(out), flush=True)


def run_large(args):
    """The large configurations once, outside the timed-steps contract: c4
    (plan, solve, hole filling, T(E), then the gradient of the summed T(E)
    by tsg_transmission_vjp, checked by the exact uniform-shift identity)
    and c5 on a subset of its planned windows (--window-subset).  Prints one
    JSON line with timings, per-window statistics and the checks."""
    import numpy as np
    import torch
    from paper_1606_01139_amd import Operator, PLAN_SEMICLASSICAL, default_opts, FP64, FP32_BULK
    from synth.workloads import workload
    w = workload(args.config)
    g = w.grid
    prec = FP64 if args.precision == "fp64" else FP32_BULK
    opts = default_opts(precision=prec, tol=1e-8, max_restarts=args.max_restarts)
    if args.basis:
        opts.basis = args.basis
    t0 = time.perf_counter()
    oper = Operator(g.nx, g.ny, g.nz, g.h, w.V, w.absorber.as_tuple())
    wins, erange = oper.plan_windows(w.n_windows * w.nev_per_window, w.n_windows, PLAN_SEMICLASSICAL, opts)
    t_plan = time.perf_counter() - t0
    log(f"{args.config}: planned {len(wins)} windows in {t_plan:.1f} s, E range {erange}")
    if args.window_subset:
        idx = [int(x) for x in args.window_subset.split(",")]
        wins = [wins[i] for i in idx]
        log(f"solving windows {idx} of the plan: {wins}")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    n, holes, status = oper.solve_all_partitions(wins, opts, allow_noconv=True)
    t_solve = time.perf_counter() - t0
    log(f"solve: {n} unique pairs in {t_solve:.1f} s, status {status}")
    fill = None
    if args.fill_rounds and not args.window_subset:
        t0 = time.perf_counter()
        added, rounds, n, left, st2 = oper.fill_holes(erange[0], max(k for _, k in wins), args.fill_rounds, opts,
                                                      allow_noconv=True)
        fill = {"rounds": rounds, "inserted": added, "holes_left": left, "seconds": round(time.perf_counter() - t0, 2)}
        status = max(status, st2)
        log(f"hole filling: {fill}")
    t_solve_all = t_solve + (fill["seconds"] if fill else 0.0)
    eps = oper.eigenvalues()
    E = energy_grid(eps, w.n_energies)
    t0 = time.perf_counter()
    T = oper.transmission(E)
    t_T = time.perf_counter() - t0
    nparts = len(wins) + (fill["inserted"] if fill else 0)
    stats = [oper.stats(j) for j in range(nparts)]
    out = {"config": {"workload": f"{args.config}: {g.nx}x{g.ny}x{g.nz} grid (N={g.n}), {len(w.wells)} wells, "
                                  f"{w.n_windows} windows x {w.nev_per_window} planned"
                                  + (f", windows {args.window_subset} solved" if args.window_subset else ""),
                      "precision": args.precision, "status": int(status), "e_range": [round(x, 6) for x in erange]},
           "unique_converged_eigenpairs": int(n), "plan_s": round(t_plan, 2), "solve_s": round(t_solve_all, 2),
           "eigenpairs_per_s": round(n / t_solve_all, 3), "transmission_s": round(t_T, 3),
           "n_energies": len(E), "T_max": float(np.max(T)), "T_min": float(np.min(T)), "hole_filling": fill,
           "windows": [{"shift": round(st.shift, 6), "nev": st.nev, "n_conv": st.n_conv, "restarts": st.restarts,
                        "restarts_bulk": st.restarts_bulk, "max_backward_error": st.max_backward_error,
                        "breakdowns": st.breakdowns} for st in stats]}
    if args.vjp:
        wts = np.ones(len(E))
        t0 = time.perf_counter()
        dV, dab = oper.transmission_vjp(E, wts, allow_noconv=True)
        t_vjp = time.perf_counter() - t0
        # A uniform shift of V by c moves every eigenvalue by c and keeps the
        # vectors, so T_S(E) becomes T_S(E - c): the gradient summed over the
        # grid equals -sum_e w_e dT/dE(E_e), here by central differences in E
        # on the same eigenpairs (no new solve)
        d = 1e-6 * max(1.0, float(np.abs(E).max()))
        dTdE = (oper.transmission(E + d) - oper.transmission(E - d)) / (2 * d)
        lhs, rhs = float(dV.sum()), float(-(wts * dTdE).sum())
        out["gradient"] = {"seconds": round(t_vjp, 2), "status": int(oper.vjp_status), "finite": bool(np.all(np.isfinite(dV)) and np.all(np.isfinite(dab))),
                           "dL_dabs": [float(x) for x in dab], "dL_dV_norm": float(np.linalg.norm(dV)),
                           "uniform_shift_identity": {"sum_dL_dV": lhs, "minus_sum_dT_dE": rhs,
                                                      "rel_diff": abs(lhs - rhs) / max(abs(rhs), 1e-300)}}
        log(f"gradient: {out['gradient']}")
    oper.close()
    print(json.dumps(out), flush=True)


def k4_flops(m):
    """Algorithmic real flops of one m x m complex eigen-decomposition:
    Householder Hessenberg reduction with accumulation (10/3 + 4/3 m^3) and
    the QR algorithm with Schur vectors (about 25 m^3), counted for real
    arithmetic and scaled by 4 for complex multiply-adds."""
    return 4.0 * (10.0 / 3.0 + 4.0 / 3.0 + 25.0) * m ** 3


# Bytes in and out of the L2s per launch, from the FETCH_SIZE and WRITE_SIZE
# counters, each scaled by what it reads for a plain 512 MiB copy (fetch x 2,
# write x 1); only the shapes below were measured.
K4_TRAFFIC_C2 = 76_031_485_356  # 8 x 450 x 450 complex128
STENCIL_TRAFFIC = {
    (32, 32, 64, 16, "c128"): 38_580_166,
    (64, 64, 160, 64, "c64"): 1_274_024_982,
    (64, 64, 160, 64, "c128"): 2_184_730_519,
}


def auto_basis(nev, block=2):
    """The library's automatic basis size (about 9 nev, at least 40)."""
    m = max(9 * nev, nev + 4 * block, 40)
    return ((m + block - 1) // block) * block


def k4_roofline(m, batch, reps=3):
    """Average duration of the batched small eigensolve (the dominant kernel
    family of a solve) at the solve's basis size, timed with HIP events on
    the stream the library launches on."""
    import numpy as np
    import torch
    from paper_1606_01139_amd import dense_eig
    rng = np.random.default_rng(7)
    Hs = []
    for _ in range(batch):
        X = rng.standard_normal((m, m)) + 1j * rng.standard_normal((m, m))
        # Rayleigh-Ritz-like: Hermitian part plus a small negative-imaginary part
        Hs.append((X + X.conj().T) / 2 - 0.05j * (X @ X.conj().T) / m)
    H0 = torch.tensor(np.stack(Hs), device="cuda")
    st = torch.cuda.current_stream()
    H = H0.clone()
    dense_eig(H)  # first call loads the kernels
    ms = []
    for _ in range(reps):
        H = H0.clone()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        e0.record(st)
        dense_eig(H)
        e1.record(st)
        torch.cuda.synchronize()
        ms.append(e0.elapsed_time(e1))
    avg = sum(ms) / len(ms)
    fl = k4_flops(m) * batch
    tf = fl / (avg * 1e-3) / 1e12
    traffic = K4_TRAFFIC_C2 if (m, batch) == (450, 8) else None
    return {"bound": "alu", "achieved": round(tf, 5), "peak": FP64_PEAK_TFLOPS, "unit": "TFLOP/s",
            "frac": round(tf / FP64_PEAK_TFLOPS, 6), "traffic": traffic,
            "kernel": "K4 small eigensolve: hess_slab_p/u_kernel (Hessenberg, row slabs over several "
                      "workgroups per window; hessenberg_kernel below m = 192) + householder_z_kernel + "
                      "schur_kernel + hreplay_kernel + zreplay_kernel + trevc_kernel + small_gemm_kernel + colnorm_kernel",
            "launch": f"{batch} windows x {m}x{m} complex128", "avg_ms": round(avg, 3),
            "algorithmic_flops": fl}


def stencil_roofline(nx, ny, nz, ncols, dtype, reps=30):
    """Average duration of the stencil kernel on N x ncols vectors, timed with
    HIP events on the stream the library launches on."""
    import numpy as np
    import torch
    from paper_1606_01139_amd import Operator
    N = nx * ny * nz
    V = np.linspace(-2.0, 0.0, N)
    oper = Operator(nx, ny, nz, 0.5, V, (0.5, 2.0, 0.0, 0.5, 2.0, (nz - 1) * 0.5))
    tdt = torch.complex128 if dtype == "c128" else torch.complex64
    X = torch.randn(ncols, N, dtype=tdt, device="cuda")
    Y = torch.empty_like(X)
    for _ in range(3):
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
    bytes_alg = 2 * N * ncols * s_c + N * s_r + nz * s_r
    gbs = bytes_alg / (ms * 1e-3) / 1e9
    oper.close()
    return {"bound": "hbm", "achieved": round(gbs, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": round(gbs / HBM_PEAK_GBS, 4), "traffic": STENCIL_TRAFFIC.get((nx, ny, nz, ncols, dtype)),
            "kernel": f"stencil_kernel<{'double' if dtype == 'c128' else 'float'},6>",
            "launch": f"{nx}x{ny}x{nz} (N={N}) x {ncols} cols", "avg_ms": round(ms, 5),
            "algorithmic_bytes": bytes_alg}


CPU_SAMPLE_NEV = 10
CPU_LOWEST_NEV = 40


def _cpu_worker(conn, config):
    """Child process (started before the parent touches the GPU): builds the
    oracle's operator of `config`, then for each job (kind, shift, nev,
    threads) times the oracle with BLAS limited to `threads` threads on
    either the nev eigenpairs of lowest real part ("lowest": ARPACK 'SR', the
    exterior end where the partitioned interval starts) or the nev nearest
    `shift` ("window": ARPACK 'SM' on the shifted operator), and sends back
    (status, seconds, pairs)."""
    try:
        from threadpoolctl import threadpool_limits
        from oracle import operator as op, eigen
        from synth.workloads import workload
        w = workload(config)
        g = w.grid
        gL, gR = op.gamma_fields(g.nx, g.ny, g.nz, g.h, w.absorber.as_tuple())
        A = op.assemble_sparse(g.nx, g.ny, g.nz, g.h, w.V, gL, gR)
    except Exception as exc:
        conn.send(("error", repr(exc), 0))
        return
    while True:
        job = conn.recv()
        if job is None:
            return
        kind, shift, nev, threads = job
        try:
            with threadpool_limits(limits=threads):
                t0 = time.perf_counter()
                if kind == "lowest":
                    e = eigen.lowest_real(A, nev)
                else:
                    e, _ = eigen.window_arpack(A, shift, nev)
                dt = time.perf_counter() - t0
            conn.send(("ok", dt, len(e)))
        except Exception as exc:  # reported in the JSON line
            conn.send(("error", repr(exc), 0))


class CpuSample:
    """The oracle timed on the host cores in a child process started before
    the GPU is touched.  Its single-thread run overlaps the GPU steps (it
    needs one core; the GPU steps need one host thread)."""

    def __init__(self, config):
        import multiprocessing as mp
        ctx = mp.get_context("spawn")
        self.conn, child = ctx.Pipe()
        self.proc = ctx.Process(target=_cpu_worker, args=(child, config), daemon=True)
        self.proc.start()
        self.t_job = None

    def start(self, kind, shift, nev, threads):
        self.job = (kind, shift, nev, threads)
        self.t_job = time.perf_counter()
        try:
            self.conn.send(self.job)
        except (BrokenPipeError, OSError):
            pass  # the worker ended early; result() reports what it sent

    def result(self, deadline):
        """Result of the started job, waiting until `deadline` (perf_counter
        seconds) at most; an unfinished run ends the worker."""
        kind, shift, nev, threads = self.job
        ready = False
        while True:  # a progress line every 30 s while the oracle runs
            left = deadline - time.perf_counter()
            if self.conn.poll(max(min(left, 30.0), 0.0)):
                ready = True
                break
            if left <= 30.0:
                break
            log(f"oracle {kind} sample still running ({time.perf_counter() - self.t_job:.0f} s, {threads} threads)")
        if ready:
            kind, dt, n = self.conn.recv()
            if kind == "ok":
                return {"seconds": round(dt, 2), "eigenpairs": n, "value": round(n / dt, 4), "threads": threads}
            return {"error": dt, "threads": threads}
        waited = time.perf_counter() - self.t_job
        self.close()
        return {"unfinished_after_s": round(waited, 1), "threads": threads,
                "value_upper_bound": round(nev / waited, 4)}

    def close(self):
        if self.proc.is_alive():
            try:
                self.conn.send(None)
            except Exception:
                pass
            self.proc.join(2)
        if self.proc.is_alive():
            self.proc.kill()
            self.proc.join(5)


def cpu_baseline_line(single, multi, window, config, nev, shift):
    """cpu_baseline object: the single-thread run (primary), the all-core
    run, and the interior-window attempt (when it ran)."""
    prim = single or {}
    val = prim.get("value", prim.get("value_upper_bound"))
    out = {"value": val, "unit": "eigenpairs/s", "cores": 1, "kind": "oracle",
           "sample": f"the {nev} eigenpairs of lowest real part of the {config} operator (the bottom of the same "
                     f"combined set the GPU step returns), by the oracle's ARPACK 'SR' (scipy, FP64), BLAS limited to "
                     f"one thread; interior windows cost the oracle far more per pair (see interior_window)"}
    if "unfinished_after_s" in prim:
        out["sample"] += f"; not finished after {prim['unfinished_after_s']} s, so value is an upper bound"
    if "error" in prim:
        out["sample"] += f"; the run failed: {prim['error']}"
    out["single_thread"] = single
    out["all_cores"] = multi
    if window is not None:
        window = dict(window)
        window["what"] = (f"{CPU_SAMPLE_NEV} eigenpairs nearest {shift:.4f} Ha (the median planned window), ARPACK "
                          f"'SM' on the shifted operator, one thread, run beside the GPU steps")
    out["interior_window"] = window
    return out


def run_budgeted(w, opts, args, label, deadline_warm, deadline_timed):
    """Warm-up steps while fewer than args.warmup have run and the next one
    (estimated by the last) ends before deadline_warm; then timed steps while
    fewer than args.steps have run and the next ends before deadline_timed
    (at least one).  Returns (seconds, converged pairs, steps timed, warm-up
    steps run, last step's results)."""
    import torch
    p, nev = w.n_windows, w.nev_per_window
    n_r = p * nev
    est = None
    nwarm = 0
    while nwarm < args.warmup:
        if est is not None and time.perf_counter() + est > deadline_warm:
            break
        t0 = time.perf_counter()
        r = run_step(w, n_r, p, opts, args.max_windows or None, args.plan, args.fill_rounds)
        torch.cuda.synchronize()
        est = time.perf_counter() - t0
        nwarm += 1
        log(f"{label} warm-up step {nwarm} done in {est:.1f} s, n={r[1]}")
        r[0].close()
        if est is not None and time.perf_counter() + est > deadline_warm:
            break
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    total = 0
    steps = 0
    last = None
    while steps < max(args.steps, 1):
        if steps > 0 and time.perf_counter() + (time.perf_counter() - t0) / steps > deadline_timed:
            break
        r = run_step(w, n_r, p, opts, args.max_windows or None, args.plan, args.fill_rounds)
        total += r[1]
        steps += 1
        if last is not None:
            last[0].close()
        last = r
        torch.cuda.synchronize()
        log(f"{label} timed step {steps}: {time.perf_counter() - t0:.2f} s cumulative, n={r[1]}")
    torch.cuda.synchronize()
    return time.perf_counter() - t0, total, steps, nwarm, last


def main():
    t_launch = time.perf_counter()
    ap = argparse.ArgumentParser(description=__doc__)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=1,
                    help="timed steps at most; steps that would end past the wall budget are not started")
    ap.add_argument("--warmup", type=int, default=0, help="warm-up steps at most, under the same budget")
    ap.add_argument("--budget", type=float, default=420.0,
                    help="wall-clock seconds from start by which the JSON line is printed (steps are sized to it)")
    ap.add_argument("--timed-budget", type=float, default=75.0,
                    help="seconds of timed steps at most (at least one step is timed)")
    ap.add_argument("--config", default="c2")
    ap.add_argument("--precision", default="fp64", choices=["fp64", "bulk"])
    ap.add_argument("--no-compare-bulk", dest="compare_bulk", action="store_false",
                    help="skip the steps in the other precision mode (by default they run after the timed "
                         "steps, beside the oracle's interior-window sample, for the FP32-bulk speedup)")
    ap.add_argument("--max-restarts", type=int, default=2000)
    ap.add_argument("--max-windows", type=int, default=0)
    ap.add_argument("--plan", default="semiclassical", choices=["semiclassical", "sampled", "alg1"])
    ap.add_argument("--fill-rounds", type=int, default=4,
                    help="rounds of Algorithm 1's hole-filling loop after the planned windows (0: off)")
    ap.add_argument("--block", type=int, default=0)
    ap.add_argument("--basis", type=int, default=0)
    ap.add_argument("--keep", type=int, default=0)
    ap.add_argument("--groups", type=int, default=0, help="window groups iterating concurrently (0: library default)")
    ap.add_argument("--bulk-tol", type=float, default=0.0,
                    help="FP32-bulk: backward error at which the complex64 phase hands over (0: library default)")
    ap.add_argument("--extraction", default="ritz", choices=["ritz", "harmonic"],
                    help="Ritz or harmonic Ritz pairs for the window shifts")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--k4-only", action="store_true",
                    help="time only the batched small eigensolve at the solve's shape and print its roofline object")
    ap.add_argument("--n-sys", type=int, default=64, help="systems of the ragged batch (config c3)")
    ap.add_argument("--stencil-only", action="store_true",
                    help="time only the stencil launches the line reports (with a known-size copy for the counters)")
    ap.add_argument("--large", action="store_true",
                    help="c4/c5 once: plan, solve, T(E) (and --vjp), with per-window statistics")
    ap.add_argument("--window-subset", default="", help="with --large: comma-separated indices of planned windows")
    ap.add_argument("--vjp", action="store_true", help="with --large: also the gradient of the summed T(E)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {args.gpus}): windows are independent and "
              "would be dealt across GPUs, but this benchmark measures the one-GPU share", file=sys.stderr)
        sys.exit(2)
    cpu = None
    if not (args.no_cpu_baseline or args.k4_only or args.stencil_only or args.large or args.config == "c3"):
        cpu = CpuSample(args.config)  # before this process touches the GPU
    import torch
    from paper_1606_01139_amd import default_opts, FP64, FP32_BULK
    from synth.workloads import workload

    torch.cuda.set_device(0)
    if args.k4_only:
        w = workload(args.config)
        out = {"roofline": k4_roofline(args.basis or auto_basis(w.nev_per_window), w.n_windows)}
        # a plain device copy of known size, the reference for HBM byte counters
        nb = 512 << 20
        x = torch.ones(nb // 8, dtype=torch.float64, device="cuda")
        y = torch.empty_like(x)
        y.copy_(x)
        torch.cuda.synchronize()
        out["calibration_copy_bytes"] = nb
        print(json.dumps(out), flush=True)
        return
    if args.stencil_only:
        w = workload(args.config)
        g = w.grid
        out = {"stencil": [stencil_roofline(g.nx, g.ny, g.nz, 2 * w.n_windows, "c128"),
                           stencil_roofline(64, 64, 160, 64, "c64"), stencil_roofline(64, 64, 160, 64, "c128")]}
        nb = 512 << 20
        x = torch.ones(nb // 8, dtype=torch.float64, device="cuda")
        y = torch.empty_like(x)
        y.copy_(x)
        torch.cuda.synchronize()
        out["calibration_copy_bytes"] = nb
        print(json.dumps(out), flush=True)
        return
    if args.config == "c3":
        run_batch(args)
        return
    if args.large:
        run_large(args)
        return
    w = workload(args.config)
    prec = FP64 if args.precision == "fp64" else FP32_BULK

    def make_opts(pr):
        o = default_opts(precision=pr, tol=1e-8, max_restarts=args.max_restarts)
        if args.block:
            o.block = args.block
        if args.basis:
            o.basis = args.basis
        if args.keep:
            o.keep = args.keep
        if args.groups:
            o.groups = args.groups
        o.extraction = 1 if args.extraction == "harmonic" else 0
        if args.bulk_tol > 0:
            o.bulk_tol = args.bulk_tol
        return o

    opts = make_opts(prec)
    nev = w.nev_per_window
    b = opts.block
    m = opts.basis or auto_basis(nev, b)
    g = w.grid
    # kernel rooflines first: they take seconds and must be in the line
    log("timing the small eigensolve and the stencil")
    roof = k4_roofline(m, w.n_windows)
    sdt = "c128" if prec == FP64 else "c64"
    stencil = [stencil_roofline(g.nx, g.ny, g.nz, b * w.n_windows, sdt),
               stencil_roofline(64, 64, 160, 64, "c64"), stencil_roofline(64, 64, 160, 64, "c128")]
    # the oracle's single-thread sample runs beside the GPU steps, on a
    # window of the same plan (the median planned shift)
    cpu_shift = None
    if cpu is not None:
        from paper_1606_01139_amd import Operator, PLAN_SEMICLASSICAL
        o0 = Operator(g.nx, g.ny, g.nz, g.h, w.V, w.absorber.as_tuple())
        wins0, _ = o0.plan_windows(w.n_windows * nev, w.n_windows, PLAN_SEMICLASSICAL, opts)
        o0.close()
        cpu_shift = sorted(s for s, _ in wins0)[len(wins0) // 2]
        cpu.start("lowest", 0.0, CPU_LOWEST_NEV, 1)
    deadline = t_launch + args.budget
    # the other-precision comparison and the oracle's all-core run need room after the timed steps
    reserve = 60.0 if cpu is not None else 0.0
    share = 0.5 if args.compare_bulk else 1.0
    t_now = time.perf_counter()
    gpu_window = max(deadline - reserve - t_now, 0.0) * share
    deadline_warm = t_now + min(0.3 * gpu_window, 0.5 * args.timed_budget)
    deadline_timed = min(t_now + gpu_window, deadline_warm + args.timed_budget)
    dt, total, steps, nwarm, last = run_budgeted(w, opts, args, args.precision, deadline_warm, deadline_timed)
    oper, n, holes, status, wins, erange, stats, T = last
    out = {
        "metric": "converged eigenpairs/s at rel. residual 1e-8",
        "value": round(total / dt, 3),
        "unit": "eigenpairs/s",
        "n_gpus": 1,
        "steps": steps,
        "warmup": nwarm,
        "ms_per_step": round(dt / steps * 1e3, 2),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64" if prec == FP64 else "c64+f64",
        "data": "synthetic",
        "config": {"workload": f"{args.config}: {g.nx}x{g.ny}x{g.nz} grid (N={g.n}), {len(w.wells)} Gaussian wells, "
                               f"{len(wins)} windows x {nev} eigenpairs, T(E) at {w.n_energies} energies",
                   "precision": args.precision, "unique_converged_eigenpairs": n, "holes_planned": holes,
                   "hole_filling": oper.fill,
                   "status": int(status), "e_range": [round(x, 6) for x in erange],
                   "planner": args.plan, "plan_seconds_last_step": round(oper.plan_seconds, 3),
                   "block": b, "basis": m, "groups": opts.groups, "extraction": args.extraction,
                   "steps_requested": args.steps, "warmup_requested": args.warmup,
                   "budget_s": args.budget},
        "roofline": roof,
        "stencil": stencil,
        "windows": [{"shift": round(s.shift, 6), "nev": s.nev, "n_conv": s.n_conv, "restarts": s.restarts,
                     "restarts_bulk": s.restarts_bulk, "matvecs": s.matvecs,
                     "max_backward_error": s.max_backward_error} for s in stats],
    }
    oper.close()
    single = multi = window = None
    window_started = False
    if cpu is not None:
        log("waiting for the oracle's single-thread sample")
        single = cpu.result(deadline - 0.5 * reserve)
        if "value" in single:
            ncpu = len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else (os.cpu_count() or 1)
            threads = max(1, min(ncpu, int(os.environ.get("OMP_NUM_THREADS", ncpu))))
            if single["seconds"] < deadline - time.perf_counter() - 10.0:
                log(f"timing the oracle's all-core sample ({threads} threads)")
                cpu.start("lowest", 0.0, CPU_LOWEST_NEV, threads)
                multi = cpu.result(deadline - 5.0)
            left = deadline - time.perf_counter() - 5.0
            if "value" in (multi or {}) and left > 20.0:
                # one thread, beside the other-precision steps on the GPU
                log(f"the oracle on an interior window for {left:.0f} s at most")
                cpu.start("window", cpu_shift, CPU_SAMPLE_NEV, 1)
                window_started = True
    if args.compare_bulk:
        other = FP32_BULK if prec == FP64 else FP64
        t_now = time.perf_counter()
        left = max(deadline - 5.0 - t_now, 0.0)
        steps2 = 0
        if left > 3.0 * dt / steps:  # room for a warm-up and a timed step at about 1.5 x the time
            dt2, total2, steps2, _, last2 = run_budgeted(w, make_opts(other), args, "other precision",
                                                         t_now + 0.3 * left, t_now + left)
        if steps2:
            last2[0].close()
            t64, tb = (dt / steps, dt2 / steps2) if prec == FP64 else (dt2 / steps2, dt / steps)
            out["fp32_bulk_vs_fp64"] = {"fp64_s_per_step": round(t64, 2), "bulk_s_per_step": round(tb, 2),
                                        "speedup": round(t64 / tb, 3), "other_unique_converged": last2[1],
                                        "other_status": int(last2[3]), "other_steps": steps2}
        else:
            out["fp32_bulk_vs_fp64"] = {"skipped": "no time left in the budget for a step"}
    if cpu is not None:
        if window_started:
            window = cpu.result(deadline - 3.0)
        cpu.close()
        out["cpu_baseline"] = cpu_baseline_line(single, multi, window, args.config, CPU_LOWEST_NEV, cpu_shift)
    out["wall_s"] = round(time.perf_counter() - t_launch, 1)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
