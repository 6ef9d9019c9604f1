"""Writes tests/golden/c5_window0.json: the oracle's first planned window of
the c5 workload (64 x 64 x 160 grid, N = 655,360, 32 windows x 64 pairs),
for the GPU parity test of that window.

Calls only oracle/ (and synth/ for the seeded potential).  Steps:
  * E_min: the lowest real part, from the K lowest-real-part eigenpairs of
    the operator (ARPACK 'SR', complete below the largest real part
    returned);
  * planned windows: n_r = 2,048 split equally over p = 32 partitions,
    shifts from the semiclassical counting function (the planner's
    reading); only the first is used;
  * the window: the 64 eigenvalues nearest its shift (Eq. (3)), valid only
    when its disk of radius |eps_64 - sigma| lies below the real part up to
    which the computed set is complete (checked, or the script fails).

Run once (about ten minutes on 4 cores):  python tests/golden/make_c5_window0.py
"""
from __future__ import annotations

import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

from oracle import eigen, operator as op, partition  # noqa: E402
from synth.workloads import workload  # noqa: E402

K_LOWEST = 90


def main():
    w = workload("c5")
    g = w.grid
    ab = w.absorber.as_tuple()
    gL, gR = op.gamma_fields(g.nx, g.ny, g.nz, g.h, ab)
    A = op.assemble_sparse(g.nx, g.ny, g.nz, g.h, w.V, gL, gR)
    t0 = time.time()
    eps_all, _, e_trust = eigen.lowest_real_pairs(A, K_LOWEST)
    print(f"lowest {K_LOWEST} eigenvalues in {time.time() - t0:.0f} s, complete below Re = {e_trust:.6f}", flush=True)
    e_min = float(eps_all[0].real)
    counts = partition.equal_counts(w.n_windows * w.nev_per_window, w.n_windows)
    shifts = partition.semiclassical_windows(w.V, g.h, (g.nx, g.ny, g.nz), e_min, counts)
    sigma, nev = float(shifts[0]), int(counts[0])
    order = eigen.order_nearest(eps_all, sigma)
    d = np.abs(eps_all[order] - sigma)
    radius = float(d[nev - 1])
    if sigma + radius >= e_trust:
        raise SystemExit(f"window radius {radius} reaches beyond the complete set (Re < {e_trust}); raise K_LOWEST")
    win = eps_all[order[:nev]]
    win = win[np.lexsort((win.imag, win.real))]
    out = {
        "workload": "c5: 64x64x160 grid, 64 wells, 32 windows x 64 eigenpairs; first planned window",
        "e_min": e_min,
        "e_trust": e_trust,
        "shift": sigma,
        "nev": nev,
        "gap_at_edge": float(d[nev] - d[nev - 1]),
        "re": [float(x) for x in win.real],
        "im": [float(x) for x in win.imag],
    }
    path = os.path.join(HERE, "c5_window0.json")
    with open(path, "w") as f:
        json.dump(out, f, indent=1)
    print(f"wrote {path}: shift {sigma:.10f}, radius {radius:.6f}, gap at the edge {out['gap_at_edge']:.3e}")


if __name__ == "__main__":
    main()
