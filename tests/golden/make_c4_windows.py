"""Writes tests/golden/c4_windows.json: the oracle's first two planned windows
of the c4 workload (48 x 48 x 96 grid, N = 221,184, 12 windows x 40 pairs),
for the GPU parity test of those windows and of the gradient on them.

Calls only oracle/ (and synth/ for the seeded potential).  Steps:
  * E_min: the lowest real part, from the K lowest-real-part eigenpairs of
    the operator (ARPACK 'SR', complete below the largest real part
    returned);
  * planned windows: n_r = 480 split equally over p = 12 partitions, shifts
    from the semiclassical counting function (the planner's reading); the
    first two are used;
  * each window: the 40 eigenvalues nearest its shift (Eq. (3)), valid only
    when its disk lies below the real part up to which the computed set is
    complete (checked, or the script fails);
  * Algorithm 2 over the two windows (the combined set the test compares).

Run once (about ten minutes on 6 cores):  python tests/golden/make_c4_windows.py
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

K_LOWEST = 130
N_WIN = 2


def main():
    w = workload("c4")
    g = w.grid
    ab = w.absorber.as_tuple()
    gL, gR = op.gamma_fields(g.nx, g.ny, g.nz, g.h, ab)
    A = op.assemble_sparse(g.nx, g.ny, g.nz, g.h, w.V, gL, gR)
    nrm = op.gershgorin_norm(g.h, w.V, (gL + gR).max())
    t0 = time.time()
    eps_all, U_all, e_trust = eigen.lowest_real_pairs(A, K_LOWEST)
    print(f"lowest {K_LOWEST} pairs in {time.time() - t0:.0f} s, complete below Re = {e_trust:.6f}", flush=True)
    e_min = float(eps_all[0].real)
    counts = partition.equal_counts(w.n_windows * w.nev_per_window, w.n_windows)
    shifts = partition.semiclassical_windows(w.V, g.h, (g.nx, g.ny, g.nz), e_min, counts)
    windows, parts = [], []
    for j in range(N_WIN):
        sigma, nev = float(shifts[j]), int(counts[j])
        order = eigen.order_nearest(eps_all, sigma)
        d = np.abs(eps_all[order] - sigma)
        radius = float(d[nev - 1])
        if sigma + radius >= e_trust:
            raise SystemExit(f"window {j}: radius {radius} reaches beyond the complete set; raise K_LOWEST")
        win = eps_all[order[:nev]]
        parts.append((win, U_all[:, order[:nev]]))
        windows.append({"shift": sigma, "nev": nev, "gap_at_edge": float(d[nev] - d[nev - 1]),
                        "re": [float(x) for x in win.real], "im": [float(x) for x in win.imag]})
    comb = partition.combine(parts, nrm)
    out = {
        "workload": "c4: 48x48x96 grid, 24 wells, 12 windows x 40 eigenpairs; first two planned windows",
        "e_min": e_min,
        "e_trust": e_trust,
        "windows": windows,
        "combined": {"re": [float(x) for x in comb.eps.real], "im": [float(x) for x in comb.eps.imag]},
    }
    path = os.path.join(HERE, "c4_windows.json")
    with open(path, "w") as f:
        json.dump(out, f, indent=1)
    print(f"wrote {path}: shifts {[round(x['shift'], 8) for x in windows]}, combined {len(comb.eps)}")


if __name__ == "__main__":
    main()
