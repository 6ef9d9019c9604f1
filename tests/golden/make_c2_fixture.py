"""Writes tests/golden/c2_reference.json: the oracle's result for the c2
workload in the benchmark's configuration, for the full-set GPU parity test.

Calls only oracle/ (and synth/ for the seeded potential).  Steps, as the
method defines the result:
  * E_min: the lowest real part (exterior solve); E_max: the bound
    max V + 3 max|symbol| / (2 h^2) on the real parts;
  * planned windows: n_r = 400 split equally over p = 8 partitions, shifts
    from the semiclassical counting function (the planner's reading);
  * each window: the n_{r,j} eigenpairs nearest its shift (Eq. (3)), taken
    from the K lowest-real-part eigenpairs of the operator (ARPACK 'SR'); a
    window is valid only when its disk of radius |eps_n - sigma| lies below
    the real part up to which that set is complete;
  * Algorithm 2 and Algorithm 1's hole-filling loop (4 rounds at most,
    inserted counts capped at the planned 50);
  * T(E) at 200 energies spread over the real parts of the combined set.

Run once (about half an hour on 4 cores):  python tests/golden/make_c2_fixture.py
"""
from __future__ import annotations

import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

from oracle import eigen, operator as op, partition, transport  # noqa: E402
from synth.workloads import workload  # noqa: E402

K_LOWEST = 470
N_CAP = 50
ROUNDS = 4


def main():
    w = workload("c2")
    g = w.grid
    ab = w.absorber.as_tuple()
    gL, gR = op.gamma_fields(g.nx, g.ny, g.nz, g.h, ab)
    A = op.assemble_sparse(g.nx, g.ny, g.nz, g.h, w.V, gL, gR)
    nrm = op.gershgorin_norm(g.h, w.V, (gL + gR).max())
    t0 = time.time()
    eps_all, U_all, e_trust = eigen.lowest_real_pairs(A, K_LOWEST)
    print(f"lowest {K_LOWEST} pairs in {time.time() - t0:.0f} s, complete below Re = {e_trust:.6f}", flush=True)
    e_min = float(eps_all[0].real)
    e_max = float(np.max(w.V)) + op.kinetic_upper_bound(g.h)
    counts = partition.equal_counts(w.n_windows * w.nev_per_window, w.n_windows)
    shifts = partition.semiclassical_windows(w.V, g.h, (g.nx, g.ny, g.nz), e_min, counts)
    margins = []

    def solve(shift, nev):
        e, U = eigen.window_from_spectrum(eps_all, U_all, shift, nev)
        d = np.sort(np.abs(eps_all - shift))
        radius = float(d[nev - 1])
        if shift + radius >= e_trust:
            raise RuntimeError(f"window at {shift} (radius {radius}) reaches beyond the complete set ({e_trust})")
        margins.append({"shift": shift, "nev": nev, "gap_to_next": float(d[nev] - d[nev - 1])})
        return e, U

    planned = [(float(s), int(c)) for s, c in zip(shifts, counts)]
    comb, wins, rounds = partition.solve_with_hole_filling(solve, planned, nrm, e_min, e_max, g.n, N_CAP, ROUNDS)
    E = transport.energy_grid(comb.eps, w.n_energies)
    T = transport.transmission_spectral(comb.eps, comb.U, gL, gR, E)
    per_window = []
    for s, c in wins:
        e, _ = eigen.window_from_spectrum(eps_all, U_all, s, c)
        per_window.append({"shift": s, "nev": c, "re": e.real.tolist(), "im": e.imag.tolist()})
    inserted = [wd for wd in wins if wd not in planned]
    out = {
        "what": "oracle result for c2 (32x32x64, 16 wells, seed 2000) in the benchmark's configuration",
        "script": "tests/golden/make_c2_fixture.py",
        "k_lowest": K_LOWEST, "complete_below": e_trust,
        "e_min": e_min, "e_max": e_max, "norm_a": nrm,
        "planned": [{"shift": s, "nev": c} for s, c in planned],
        "inserted": [{"shift": s, "nev": c} for s, c in inserted],
        "rounds": rounds,
        "holes_left": [bool(x) for x in comb.holes],
        "windows": per_window,
        "selection_margins": margins,
        "combined": {"re": comb.eps.real.tolist(), "im": comb.eps.imag.tolist()},
        "energies": E.tolist(),
        "transmission": T.tolist(),
    }
    with open(os.path.join(HERE, "c2_reference.json"), "w") as f:
        json.dump(out, f, indent=1)
    print(f"{len(comb.eps)} combined pairs, {len(inserted)} inserted partitions in {rounds} rounds; "
          f"smallest selection margin {min(m['gap_to_next'] for m in margins):.3e}", flush=True)


if __name__ == "__main__":
    main()
