"""Spectral partitioning: Algorithm 1 (window counts and shifts) and
Algorithm 2 (combine partitions, remove redundancies, test for holes).

Test infrastructure only (see oracle/__init__.py).

Readings where the paper is silent or garbled:
  * round() is half away from zero ("standard rounding", Section 2.2);
  * for odd p the middle partition of Algorithm 1 refers to itself; it gets
    ceil(ceil(2 n_r / p) / 2);
  * Algorithm 1's E_{S,0} and n_{r,0} are E_min and 0, so that
    E_{S,1} = E_min + Delta n_{r,1} / 2 (the interval-midpoint practice of
    Section 3);
  * Algorithm 2's equality test is |lambda_m - lambda_k| <= tau with
    tau = 1e-6 ||A||_G; the projection uses the unconjugated product
    (v_k -= v_m (v_m^T v_k), v_m already c-normalised); a pair is removed
    when ||v_k||_2 after the projections is below 1e-3 of its value before,
    and kept pairs are c-normalised (u^T u = 1) rather than scaled by |v_k|,
    because the transport formula needs U^T U = I;
  * the garbled flag index holes_{k-1} is read as the interfaces between the
    partitions that own lambda_m and lambda_k: when they are adjacent, the one
    interface between them; when they are not, every interface between them,
    since two windows that share an eigenvalue overlap, so the partitions
    ordered between them cannot hide a gap (without this, a small window
    between two wide ones stays flagged although its neighbours overlap);
  * E_max (Algorithm 1's upper extremal eigenvalue) is taken as the exact
    upper bound on the real parts, max V + 3 max|symbol| / (2 h^2), instead of
    a second exterior solve: Re eps = u^H (K + V) u / u^H u lies below it;
  * the semiclassical planner estimates the counting function (how many
    eigenvalues have real part below E) from the phase-space volume of the
    Hamiltonian H = p^2/2 + V(r) over the box, with the Dirichlet surface
    correction of Weyl's asymptotics: N(E) = sum_r w k_r^3/(6 pi^2) -
    S <k_r^2>/(16 pi) with k_r^2 = 2 max(E - V(r), 0), w the volume per grid
    point, S the box surface and <.> the mean over grid points; windows sit
    at the midpoints of consecutive intervals of n_{r,j} estimated
    eigenvalues, as in the density-sampling planner below;
  * density sampling (Section 2.2, "a few eigenpairs at several sample
    points") is read as: 8 eigenpairs nearest each of S = max(2p, 8) shifts
    spread evenly over [E_min, top], each giving a local density
    (8 - 1)/(spread of their real parts) at the mean of their real parts;
    the piecewise-linear density is integrated from E_min into a counting
    function, and window j is centred between the points where it reaches
    n_{r,1} + ... + n_{r,j-1} and n_{r,1} + ... + n_{r,j} (the interval
    midpoints of Section 3); beyond the last sample the last density is
    extended.  The region's top is guessed from the free-particle counting
    function of the box (Weyl's law), which only decides where to sample;
  * the repeat loop of Algorithm 1 (hole filling) orders the partitions by
    shift, so that interface j lies between partitions j and j+1; the gap of
    a flagged interface is min Re of the upper partition's eigenvalues minus
    max Re of the lower one's; the inserted count n = ceil(3/2 gap / Delta)
    with Delta = (E_max - E_min)/N is clamped to [1, n_cap], n_cap being the
    largest planned n_{r,j}: Delta is a mean over the whole spectrum, so at
    its low end, where eigenvalues are sparser than the mean, the formula
    asks for far more than one window holds, and the loop repeats instead.
    The loop stops when no flag is left or after a given number of rounds.
    The partitioned interval starts at E_min, itself an eigenvalue (found by
    the exterior solve); the loop treats it as a partition of one pair below
    the first window, so when the lowest computed real part lies more than
    Algorithm 2's tau above E_min, that gap is a hole like the others (a
    first window placed where the spectrum is sparse need not reach down to
    E_min).
"""
from __future__ import annotations

import math
from dataclasses import dataclass
from typing import List, Sequence, Tuple

import numpy as np

from .eigen import order_real


def round_half_away(x: float) -> int:
    return int(math.floor(abs(x) + 0.5)) * (1 if x >= 0 else -1)


def alg1_counts(n_r: int, p: int) -> List[int]:
    """n_{r,j} of Algorithm 1: fewer eigenpairs for partitions deeper in the
    spectrum; n_{r,j} + n_{r,p-j+1} = ceil(2 n_r / p)."""
    if p < 1 or n_r < 1:
        raise ValueError("need p >= 1 and n_r >= 1")
    counts = [0] * (p + 1)  # 1-based
    top = math.ceil(2 * n_r / p)
    for j in range(1, p + 1):
        if j <= p / 2:
            counts[j] = round_half_away(2.0 / (1.5 + (j - 1) / p) * n_r / p)
    for j in range(1, p + 1):
        if j > p / 2:
            mirror = p - j + 1
            if mirror == j:
                counts[j] = math.ceil(top / 2)
            else:
                counts[j] = top - counts[mirror]
    return counts[1:]


def equal_counts(n_r: int, p: int) -> List[int]:
    base = n_r // p
    return [base + (1 if j < n_r - base * p else 0) for j in range(p)]


def alg1_shifts(counts: Sequence[int], e_min: float, e_max: float, n: int) -> List[float]:
    """E_{S,j} = E_{S,j-1} + ((E_max - E_min)/N) (n_{r,j} + n_{r,j-1}) / 2."""
    delta = (e_max - e_min) / n
    shifts = []
    prev_s, prev_n = e_min, 0
    for c in counts:
        s = prev_s + delta * (c + prev_n) / 2.0
        shifts.append(s)
        prev_s, prev_n = s, c
    return shifts


def sample_shifts(e_min: float, n_r: int, p: int, box_lengths, n_samples: int = 0) -> List[float]:
    """Sample shifts of the density-sampling planner (see module notes)."""
    lx, ly, lz = box_lengths
    kf = (6.0 * math.pi ** 2 * n_r / (lx * ly * lz)) ** (1.0 / 3.0)
    top = max(0.5 * kf * kf, 0.0)
    top = max(top, e_min + 0.25) * 1.25 + 0.25 * abs(e_min)
    S = n_samples or max(2 * p, 8)
    return [e_min + (top - e_min) * (i + 0.5) / S for i in range(S)]


def sampled_windows(e_min: float, samples: Sequence[np.ndarray], counts: Sequence[int]) -> List[float]:
    """Window shifts from sampled eigenvalues (each entry: the eigenvalues
    nearest one sample shift)."""
    pc = [e_min]
    rho = [0.0]
    for ev in samples:
        re = np.sort(np.asarray(ev).real)
        pc.append(float(re.mean()))
        rho.append((len(re) - 1) / max(float(re[-1] - re[0]), 1e-12))
    rho[0] = rho[1]
    order = sorted(range(len(pc)), key=lambda i: pc[i])
    xs = [pc[order[0]]]
    cum = [0.0]
    for q in range(1, len(order)):
        x0, x1 = pc[order[q - 1]], pc[order[q]]
        xs.append(x1)
        cum.append(cum[-1] + 0.5 * (rho[order[q - 1]] + rho[order[q]]) * (x1 - x0))

    def inverse(target):
        for q in range(1, len(xs)):
            if cum[q] >= target:
                f = (target - cum[q - 1]) / max(cum[q] - cum[q - 1], 1e-300)
                return xs[q - 1] + f * (xs[q] - xs[q - 1])
        return xs[-1] + (target - cum[-1]) / max(rho[order[-1]], 1e-12)

    shifts, acc = [], 0.0
    for c in counts:
        shifts.append(0.5 * (inverse(acc) + inverse(acc + c)))
        acc += c
    return shifts


def imaginary_bands(real_windows: Sequence[Tuple[float, int]], gamma_max: float, q: int) -> List[Tuple[complex, int]]:
    """Two-dimensional partitioning (Section 2's remark for strongly
    non-Hermitian operators): every real window (shift, n) becomes q windows
    at shifts shift - i gamma_max (i + 1/2)/q, i < q, which split n as evenly
    as integers allow (the larger counts first, at least 1 each).  By Eq. (5)
    the eigenvalues' imaginary parts lie in [-gamma_max, 0], so the bands
    tile that range."""
    out = []
    for shift, n in real_windows:
        base = n // q
        for i in range(q):
            cnt = max(base + (1 if i < n - base * q else 0), 1)
            out.append((complex(shift, -gamma_max * (i + 0.5) / q), cnt))
    return out


def box_lengths(shape, h: float):
    """Edges of the Dirichlet box: the grid plus one spacing (the zero
    values sit one step outside the first and last points)."""
    return tuple((n + 1) * h for n in shape)


def semiclassical_count(V: np.ndarray, h: float, shape, E: float) -> float:
    """Estimated number of eigenvalues with real part below E (module notes)."""
    lx, ly, lz = box_lengths(shape, h)
    vol = lx * ly * lz
    surf = 2.0 * (lx * ly + ly * lz + lx * lz)
    k2 = np.maximum(2.0 * (E - np.asarray(V, dtype=np.float64)), 0.0)
    return (vol / k2.size) * float(np.sum(k2 ** 1.5)) / (6.0 * math.pi ** 2) - surf * float(np.mean(k2)) / (16.0 * math.pi)


def semiclassical_windows(V: np.ndarray, h: float, shape, e_min: float, counts: Sequence[int]) -> List[float]:
    """Window shifts at the midpoints of consecutive intervals holding
    n_{r,j} eigenvalues of the semiclassical counting function."""
    def inverse(target):
        if target <= 0:
            return e_min
        lo, width = e_min, 1.0
        while semiclassical_count(V, h, shape, lo + width) < target:
            width *= 2.0
        hi = lo + width
        for _ in range(100):
            mid = 0.5 * (lo + hi)
            if semiclassical_count(V, h, shape, mid) < target:
                lo = mid
            else:
                hi = mid
        return 0.5 * (lo + hi)

    shifts, acc = [], 0
    for c in counts:
        shifts.append(0.5 * (inverse(acc) + inverse(acc + c)))
        acc += c
    return shifts


@dataclass
class Combined:
    eps: np.ndarray          # ascending real part
    U: np.ndarray            # N x n, c-normalised
    owner: np.ndarray        # partition index of each kept pair
    holes: np.ndarray        # bool, p-1 interface flags (True = hole suspected)
    removed: int


def combine(windows: Sequence[Tuple[np.ndarray, np.ndarray]], norm_a: float,
            tau_rel: float = 1e-6, drop_ratio: float = 1e-3,
            keep_lowest: int = 0) -> Combined:
    """Algorithm 2 over all computed eigenpairs, partition by partition."""
    p = len(windows)
    tau = tau_rel * norm_a
    holes = np.ones(max(p - 1, 0), dtype=bool)
    kept_eps: List[complex] = []
    kept_vec: List[np.ndarray] = []
    kept_own: List[int] = []
    removed = 0
    for j, (eps_j, U_j) in enumerate(windows):
        for i in range(len(eps_j)):
            lam = complex(eps_j[i])
            v = np.array(U_j[:, i], dtype=np.complex128, copy=True)
            before = np.linalg.norm(v)
            partners = []
            for m in range(len(kept_eps)):
                if abs(kept_eps[m] - lam) <= tau:
                    vm = kept_vec[m]
                    v = v - vm * (vm @ v)
                    partners.append(kept_own[m])
            after = np.linalg.norm(v)
            if partners and after < drop_ratio * before:
                removed += 1
                for o in partners:
                    holes[min(o, j):max(o, j)] = False
                continue
            kept_eps.append(lam)
            kept_vec.append(v / np.sqrt(v @ v))
            kept_own.append(j)
    eps = np.array(kept_eps, dtype=np.complex128)
    U = np.stack(kept_vec, axis=1) if kept_vec else np.zeros((0, 0), np.complex128)
    own = np.array(kept_own, dtype=np.int64)
    o = order_real(eps)
    eps, U, own = eps[o], U[:, o], own[o]
    if keep_lowest and len(eps) > keep_lowest:
        eps, U, own = eps[:keep_lowest], U[:, :keep_lowest], own[:keep_lowest]
    return Combined(eps, U, own, holes, removed)


def hole_fill_windows(parts_eps: Sequence[np.ndarray], holes: Sequence[bool], e_min: float,
                      e_max: float, n: int, n_cap: int, tau: float) -> List[Tuple[float, int]]:
    """One pass of Algorithm 1's repeat loop: a new partition for the gap
    between E_min and the lowest computed real part when it exceeds tau, and
    for every flagged interface between partitions j and j+1 (ordered by
    shift), centred at the middle of the gap, holding 3/2 gap / Delta
    eigenpairs (clamped, module notes)."""
    delta = (e_max - e_min) / n

    def window(lo, hi):
        gap = hi - lo
        cnt = math.ceil(1.5 * gap / delta) if gap > 0 else 1
        return (0.5 * (lo + hi), int(min(max(cnt, 1), n_cap)))

    out = []
    low = min(float(np.min(np.real(e))) for e in parts_eps if len(e))
    if low > e_min + tau:
        out.append(window(e_min, low))
    for j, flagged in enumerate(holes):
        if not flagged:
            continue
        out.append(window(float(np.max(np.real(parts_eps[j]))), float(np.min(np.real(parts_eps[j + 1])))))
    return out


def solve_with_hole_filling(solve, windows: Sequence[Tuple[float, int]], norm_a: float, e_min: float,
                            e_max: float, n: int, n_cap: int, max_rounds: int):
    """Algorithm 1's partitions followed by its repeat loop: solve the
    windows (solve(shift, nev) -> (eps, U)), combine (Algorithm 2), and while
    hole_fill_windows finds a gap (a flagged interface, or the stretch above
    E_min), insert its partitions, solve them, reorder by shift and combine
    again.
    Returns (Combined, final window list ordered by shift, rounds run)."""
    wins = sorted(((float(s), int(k)) for s, k in windows), key=lambda t: t[0])
    sols = [solve(s, k) for s, k in wins]
    comb = combine(sols, norm_a)
    rounds = 0
    tau = 1e-6 * norm_a
    while rounds < max_rounds:
        new = hole_fill_windows([e for e, _ in sols], comb.holes, e_min, e_max, n, n_cap, tau)
        if not new:
            break
        rounds += 1
        wins = wins + new
        sols = sols + [solve(s, k) for s, k in new]
        order = sorted(range(len(wins)), key=lambda i: wins[i][0])
        wins = [wins[i] for i in order]
        sols = [sols[i] for i in order]
        comb = combine(sols, norm_a)
    return comb, wins, rounds

