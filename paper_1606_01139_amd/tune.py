"""Runs the stencil autotuner (tsg_tune_stencil) on the launch shapes of the
standard workloads and writes tuning/stencil_gfx950.json, which the binding
loads into the library at start-up.

Usage (on the GPU):  python -m paper_1606_01139_amd.tune [--out PATH]

Shapes: the solver's launches on c2 (32x32x64; 2 x 8 columns per expansion
step, 50 x 8 for the residual check, 450 x 8 for the Rayleigh-Ritz
product, complex128 and complex64) and the large c5 grid (64x64x160, 64
columns, complex128 and complex64).
"""
from __future__ import annotations

import argparse
import json
import sys

from .binding import C128, C64, DEFAULT_TUNING, Operator

SHAPES = [
    ((32, 32, 64), [16, 400, 3600], [C128, C64]),
    ((64, 64, 160), [64], [C128, C64]),
]


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__)
    ap.add_argument("--out", default=DEFAULT_TUNING)
    ap.add_argument("--reps", type=int, default=10)
    args = ap.parse_args(argv)
    import numpy as np
    import torch  # the device is set up the way the rest of the package uses it
    if not torch.cuda.is_available():
        raise SystemExit("the autotuner needs a GPU")
    torch.cuda.set_device(0)
    results = []
    for (nx, ny, nz), cols_list, dtypes in SHAPES:
        V = np.linspace(-2.0, 0.0, nx * ny * nz)
        op = Operator(nx, ny, nz, 0.5, V, (0.5, 2.0, 0.0, 0.5, 2.0, (nz - 1) * 0.5))
        for cols in cols_list:
            for dt in dtypes:
                geo, us = op.tune_stencil(cols, dt, args.reps, args.out)
                results.append({"grid": [nx, ny, nz], "cols": cols, "dtype": "c128" if dt == C128 else "c64",
                                "best": geo, "us": round(us, 2)})
                print(json.dumps(results[-1]), flush=True)
        op.close()
    return 0


if __name__ == "__main__":
    sys.exit(main())
