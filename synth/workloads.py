"""Synthetic stand-ins for the paper's DFT systems.

The paper's Hamiltonians (C chain, Au(111) nanowire, BDT junction;
Section 3) come from self-consistent PARSEC runs that are not available, so
every workload here is synthetic: a uniform grid of spacing h (bohr), a local
potential made of attractive Gaussian wells, and two Gaussian absorbers in z
at the ends of the cell (the form of Eq. (1) with Gamma diagonal and Gaussian,
Section 1).  Units are Hartree and bohr.

Recipe (all draws from numpy PCG64 with the stated seed):
  * well depth  d ~ U[-5, -1] Ha, width s ~ U[0.8, 1.5] bohr,
    centre uniform in [0, (n-1) h] per axis (wire-like cells: x and y
    centres uniform in the middle third of the cell instead);
  * V(r) = sum_w d_w exp(-|r - c_w|^2 / (2 s_w^2)) at r = (i h, j h, k h);
  * absorbers: amplitude 0.5 Ha, standard deviation 2 bohr, centred on the
    first and last z planes.
"""
from __future__ import annotations

from dataclasses import dataclass, field
from typing import List, Optional, Tuple

import numpy as np

H_DEFAULT = 0.5


@dataclass(frozen=True)
class Grid:
    nx: int
    ny: int
    nz: int
    h: float = H_DEFAULT
    fd_radius: int = 6

    @property
    def n(self) -> int:
        return self.nx * self.ny * self.nz


@dataclass(frozen=True)
class Absorber:
    amp_l: float
    width_l: float
    z_l: float
    amp_r: float
    width_r: float
    z_r: float

    @staticmethod
    def ends(grid: Grid, amp: float = 0.5, width: float = 2.0) -> "Absorber":
        return Absorber(amp, width, 0.0, amp, width, (grid.nz - 1) * grid.h)

    def as_tuple(self) -> Tuple[float, ...]:
        return (self.amp_l, self.width_l, self.z_l, self.amp_r, self.width_r, self.z_r)


@dataclass
class Workload:
    name: str
    grid: Grid
    V: np.ndarray              # float64, length N, x fastest
    absorber: Absorber
    n_windows: int
    nev_per_window: int
    n_energies: int
    wells: np.ndarray = field(repr=False, default=None)  # (n_wells, 5): d, s, cx, cy, cz


def draw_wells(grid: Grid, n_wells: int, seed: int, wire: bool = False) -> np.ndarray:
    rng = np.random.Generator(np.random.PCG64(seed))
    out = np.empty((n_wells, 5))
    lx, ly, lz = (grid.nx - 1) * grid.h, (grid.ny - 1) * grid.h, (grid.nz - 1) * grid.h
    for w in range(n_wells):
        d = rng.uniform(-5.0, -1.0)
        s = rng.uniform(0.8, 1.5)
        if wire:
            cx = rng.uniform(lx / 3.0, 2.0 * lx / 3.0)
            cy = rng.uniform(ly / 3.0, 2.0 * ly / 3.0)
        else:
            cx = rng.uniform(0.0, lx)
            cy = rng.uniform(0.0, ly)
        cz = rng.uniform(0.0, lz)
        out[w] = (d, s, cx, cy, cz)
    return out


def wells_potential(grid: Grid, wells: np.ndarray) -> np.ndarray:
    x = np.arange(grid.nx) * grid.h
    y = np.arange(grid.ny) * grid.h
    z = np.arange(grid.nz) * grid.h
    V = np.zeros((grid.nz, grid.ny, grid.nx))
    for d, s, cx, cy, cz in wells:
        gx = np.exp(-((x - cx) ** 2) / (2 * s * s))
        gy = np.exp(-((y - cy) ** 2) / (2 * s * s))
        gz = np.exp(-((z - cz) ** 2) / (2 * s * s))
        V += d * gz[:, None, None] * gy[None, :, None] * gx[None, None, :]
    return V.reshape(-1).copy()


# The five workload shapes: (grid, wells, windows x eigenpairs, energies, seed, wire)
CONFIGS = {
    "c1": dict(grid=(10, 10, 20), wells=4, windows=2, nev=20, energies=50, seed=1000),
    "c2": dict(grid=(32, 32, 64), wells=16, windows=8, nev=50, energies=200, seed=2000),
    "c3": dict(grid=None, wells=None, windows=4, nev=16, energies=0, seed=3000),
    "c4": dict(grid=(48, 48, 96), wells=24, windows=12, nev=40, energies=200, seed=4000),
    "c5": dict(grid=(64, 64, 160), wells=64, windows=32, nev=64, energies=500, seed=5000, wire=True),
}


def workload(name: str, h: float = H_DEFAULT) -> Workload:
    c = CONFIGS[name]
    if c["grid"] is None:
        raise ValueError("use batch_workloads() for the ragged batch")
    g = Grid(*c["grid"], h=h)
    wells = draw_wells(g, c["wells"], c["seed"], wire=c.get("wire", False))
    return Workload(name, g, wells_potential(g, wells), Absorber.ends(g), c["windows"],
                    c["nev"], c["energies"], wells)


def small_workload(nx: int, ny: int, nz: int, n_wells: int, seed: int,
                   h: float = H_DEFAULT, amp: float = 0.5, width: float = 2.0,
                   windows: int = 2, nev: int = 8, energies: int = 16) -> Workload:
    g = Grid(nx, ny, nz, h=h)
    wells = draw_wells(g, n_wells, seed)
    return Workload(f"small{nx}x{ny}x{nz}s{seed}", g, wells_potential(g, wells),
                    Absorber.ends(g, amp, width), windows, nev, energies, wells)


def batch_workloads(n_sys: int = 64, seed: int = 3000, h: float = H_DEFAULT,
                    nxy: Tuple[int, int] = (16, 32), nzr: Tuple[int, int] = (16, 48),
                    wells: Tuple[int, int] = (4, 12)) -> List[Workload]:
    """Ragged batch: grids drawn per system, nx, ny ~ U{16..32}, nz ~ U{16..48}."""
    out = []
    c = CONFIGS["c3"]
    for s in range(n_sys):
        rng = np.random.Generator(np.random.PCG64(seed + s))
        nx = int(rng.integers(nxy[0], nxy[1] + 1))
        ny = int(rng.integers(nxy[0], nxy[1] + 1))
        nz = int(rng.integers(nzr[0], nzr[1] + 1))
        nw = int(rng.integers(wells[0], wells[1] + 1))
        g = Grid(nx, ny, nz, h=h)
        wl = draw_wells(g, nw, seed + 10_000 + s)
        out.append(Workload(f"c3.{s}", g, wells_potential(g, wl), Absorber.ends(g),
                            c["windows"], c["nev"], 0, wl))
    return out
