"""Pins for oracle.eigen (windows), oracle.partition (Algorithms 1 and 2),
oracle.transport (T(E)) and oracle.gradient (CPU only)."""
import json
import math
import os

import numpy as np
import pytest

from oracle import operator as op
from oracle import eigen, partition, transport, gradient
from synth.workloads import small_workload

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def _dense(w):
    g = w.grid
    gL, gR = op.gamma_fields(g.nx, g.ny, g.nz, g.h, w.absorber.as_tuple())
    A = op.assemble_dense(g.nx, g.ny, g.nz, g.h, w.V, gL, gR)
    return A, gL, gR


# ---------------------------------------------------------------- windows
def test_window_is_nearest_closed_form():
    # V = Gamma = 0, R = 1: the window is the n closed-form values nearest sigma
    nx, ny, nz, h = 4, 5, 7, 0.5
    z = np.zeros(nx * ny * nz)
    A = op.assemble_dense(nx, ny, nz, h, z, z, z, 1)
    one = lambda n: (1 - np.cos(np.pi * np.arange(1, n + 1) / (n + 1))) / h ** 2
    ref = (one(nx)[:, None, None] + one(ny)[None, :, None] + one(nz)[None, None, :]).ravel()
    sigma = 5.3
    eps, U = eigen.window_dense(A, sigma, 9)
    want = np.sort(ref[np.argsort(np.abs(ref - sigma))[:9]])
    np.testing.assert_allclose(np.sort(eps.real), want, atol=1e-12)


def test_window_arpack_matches_dense():
    # Tier B (ARPACK 'SM' on the shifted operator) against tier A (dense).
    w = small_workload(7, 6, 12, 3, seed=21)
    A, gL, gR = _dense(w)
    eps_all, U_all = eigen.dense_spectrum(A)
    import scipy.sparse as sp
    sigma = float(eps_all[30].real)
    e1, U1 = eigen.window_dense(A, sigma, 12)
    e2, U2 = eigen.window_arpack(sp.csr_matrix(A), sigma, 12)
    np.testing.assert_allclose(e2, e1, atol=1e-10)
    # eigenvectors agree up to sign (c-normalised)
    for k in range(12):
        d = min(np.linalg.norm(U1[:, k] - U2[:, k]), np.linalg.norm(U1[:, k] + U2[:, k]))
        assert d < 1e-7
    nrm = op.gershgorin_norm(w.grid.h, w.V, (gL + gR).max())
    for k in range(12):
        assert eigen.backward_error(A, U2[:, k], e2[k], nrm) < 1e-12


def test_lowest_real_matches_dense():
    # ARPACK 'SR' (sparse) against the dense spectrum sorted by real part
    w = small_workload(7, 6, 12, 3, seed=22)
    A, gL, gR = _dense(w)
    eps_all, _ = eigen.dense_spectrum(A)
    import scipy.sparse as sp
    got = eigen.lowest_real(sp.csr_matrix(A), 8)
    want = eps_all[np.argsort(eps_all.real)][:8]
    np.testing.assert_allclose(got, want, atol=1e-10)


def test_c_rayleigh_is_quadratic():
    w = small_workload(5, 5, 8, 2, seed=8)
    A, _, _ = _dense(w)
    eps, U = eigen.dense_spectrum(A)
    rng = np.random.default_rng(0)
    d = rng.standard_normal(A.shape[0])
    errs = []
    for t in (1e-3, 1e-4):
        u = U[:, 3] + t * d
        errs.append(abs(eigen.c_rayleigh(A, u) - eps[3]))
    assert errs[1] < errs[0] / 50  # second order: factor ~100


# ------------------------------------------------------------ Algorithm 1
def test_alg1_worked_values():
    for case in json.load(open(os.path.join(GOLD, "alg1_partitions.json")))["worked"]:
        assert partition.alg1_counts(case["n_r"], case["p"]) == case["n_rj"]


@pytest.mark.parametrize("n_r,p", [(2210, 4), (2930, 4), (3209, 2), (3209, 4), (3209, 8),
                                   (400, 8), (10, 5), (97, 7), (1, 1), (5, 3)])
def test_alg1_invariants(n_r, p):
    c = partition.alg1_counts(n_r, p)
    top = math.ceil(2 * n_r / p)
    for j in range(p):
        if j != p - 1 - j:
            assert c[j] + c[p - 1 - j] == top
    assert sum(c) >= n_r                      # Eq. (4)
    assert all(a >= b for a, b in zip(c, c[1:]))  # deeper partitions get fewer
    assert c[0] == partition.round_half_away(4 * n_r / (3 * p))


def test_alg1_against_printed_partitions():
    # The printed sizes are the formula enlarged by hand (Section 3); for the
    # four-partition runs the formula sits within 25% of every entry.  (The
    # p = 2 and p = 8 BDT rows of Table 1 were retuned further and depart by
    # up to 38%, so they pin nothing.)
    for case in json.load(open(os.path.join(GOLD, "alg1_partitions.json")))["printed"]:
        if case["p"] != 4:
            continue
        c = partition.alg1_counts(case["n_r"], case["p"])
        for a, b in zip(c, case["n_rj"]):
            assert abs(a - b) <= 0.25 * b


def test_alg1_shifts_midpoints():
    # equal counts n: shifts sit at midpoints of consecutive intervals of
    # n eigenvalues under the uniform-density estimate Delta = (Emax-Emin)/N
    s = partition.alg1_shifts([10, 10, 10], -2.0, 8.0, 100)
    np.testing.assert_allclose(s, [-2.0 + 0.1 * 5, -2.0 + 0.1 * 15, -2.0 + 0.1 * 25])
    s = partition.alg1_shifts([4, 2], 0.0, 1.0, 10)
    np.testing.assert_allclose(s, [0.2, 0.5])


# ------------------------------------------------------------ Algorithm 2
def _windows(w, shifts, nev):
    """shifts: floats, or ints meaning 'the real part of eigenvalue #i'."""
    A, gL, gR = _dense(w)
    eps_all, U_all = eigen.dense_spectrum(A)
    nrm = op.gershgorin_norm(w.grid.h, w.V, (gL + gR).max())
    shifts = [float(eps_all[s].real) if isinstance(s, int) else s for s in shifts]
    wins = [eigen.window_from_spectrum(eps_all, U_all, s, nev) for s in shifts]
    return A, gL, gR, eps_all, U_all, nrm, wins


def test_combine_duplicate_window_removed():
    w = small_workload(6, 6, 10, 3, seed=4)
    A, gL, gR, ea, Ua, nrm, wins = _windows(w, [0.5, 0.5], 10)
    c = partition.combine(wins, nrm)
    assert c.removed == 10 and len(c.eps) == 10
    assert not c.holes[0]
    np.testing.assert_allclose(c.eps, wins[0][0], atol=1e-12)


def test_combine_flags_between_overlapping_non_adjacent_windows():
    # unit vectors with eigenvalues 1..8: window 1 (between the others by
    # shift) holds only 3; windows 0 and 2 share 4, so no interface can hide
    # a gap; with window 2 moved to {6, 7} the interface 1-2 is a real gap
    N = 8
    I = np.eye(N, dtype=np.complex128)
    win = lambda ks: (np.array(ks, dtype=np.complex128), I[:, [k - 1 for k in ks]])
    c = partition.combine([win([1, 2, 3, 4]), win([3]), win([4, 5, 6])], 10.0)
    assert list(c.holes) == [False, False] and c.removed == 2 and len(c.eps) == 6
    c = partition.combine([win([1, 2, 3, 4]), win([3]), win([6, 7])], 10.0)
    assert list(c.holes) == [False, True]


def test_combine_far_windows_flag_hole():
    w = small_workload(6, 6, 10, 3, seed=4)
    A, gL, gR, ea, Ua, nrm, wins = _windows(w, [2, 60], 5)
    c = partition.combine(wins, nrm)
    assert c.removed == 0 and len(c.eps) == 10 and c.holes[0]


def test_combine_overlap_union_exact():
    # overlapping windows: the union is exactly the set of distinct eigenpairs
    w = small_workload(6, 6, 10, 3, seed=4)
    A, gL, gR, ea, Ua, nrm, wins = _windows(w, [5, 12, 19], 10)
    c = partition.combine(wins, nrm)
    ids = set()
    for e, _ in wins:
        for x in e:
            ids.add(int(np.argmin(np.abs(ea - x))))
    assert len(c.eps) == len(ids)
    np.testing.assert_allclose(np.sort_complex(c.eps), np.sort_complex(ea[sorted(ids)]), atol=1e-12)
    assert not c.holes.any()
    np.testing.assert_allclose(c.U.T @ c.U, np.eye(len(c.eps)), atol=1e-9)


def test_combine_degenerate_cluster_projector():
    # V = Gamma = 0 on a cube: threefold-degenerate levels.  Two windows
    # both holding (different bases of) the same eigenspace: combine keeps
    # exactly its dimension and the same spectral projector.
    n, h = 5, 0.5
    z = np.zeros(n ** 3)
    A = op.assemble_dense(n, n, n, h, z, z, z, 6)
    eps, U = eigen.dense_spectrum(A)
    lvl = eps[1].real  # first excited level, 3-fold
    idx = np.where(np.abs(eps.real - lvl) < 1e-9)[0]
    assert len(idx) == 3
    Q = U[:, idx]
    rng = np.random.default_rng(1)
    R = np.linalg.qr(rng.standard_normal((3, 3)))[0]   # real orthogonal mix
    wins = [(eps[idx], Q), (eps[idx], Q @ R)]
    c = partition.combine(wins, 50.0)
    assert len(c.eps) == 3 and c.removed == 3
    # basis-independent projector onto the eigenspace (eig's basis of a
    # degenerate eigenspace is not c-orthogonal; combine's output is)
    P = Q @ np.linalg.solve(Q.T @ Q, Q.T)
    np.testing.assert_allclose(c.U.T @ c.U, np.eye(3), atol=1e-10)
    np.testing.assert_allclose(c.U @ c.U.T, P, atol=1e-10)


# --------------------------------------------------------------- T(E)
def test_transmission_spectral_equals_direct_full_spectrum():
    w = small_workload(4, 4, 12, 2, seed=6)
    A, gL, gR = _dense(w)
    eps, U = eigen.dense_spectrum(A)
    E = np.linspace(eps.real.min(), eps.real.min() + 3.0, 7)
    Ts = transport.transmission_spectral(eps, U, gL, gR, E)
    Td = transport.transmission_direct(A, gL, gR, E)
    np.testing.assert_allclose(Ts, Td, rtol=1e-9, atol=1e-12)


def test_transmission_truncated_invariants():
    w = small_workload(6, 5, 12, 3, seed=9)
    A, gL, gR = _dense(w)
    eps, U = eigen.dense_spectrum(A)
    S = slice(0, 25)
    E = transport.energy_grid(eps[S], 40)
    T = transport.transmission_spectral(eps[S], U[:, S], gL, gR, E)
    assert (T >= -1e-14).all()                    # Schur product of PSD Grams
    T2 = transport.transmission_spectral(eps[S], U[:, S], gR, gL, E)
    np.testing.assert_allclose(T, T2, rtol=1e-12, atol=1e-15)   # G_S symmetric
    T0 = transport.transmission_spectral(eps[S], U[:, S], 0 * gL, gR, E)
    assert np.abs(T0).max() == 0.0


# ------------------------------------------------------------ gradient
def _pipeline_T(nx, ny, nz, h, V, absorber, shifts, nev, E):
    gL, gR = op.gamma_fields(nx, ny, nz, h, absorber)
    A = op.assemble_dense(nx, ny, nz, h, V, gL, gR)
    ea, Ua = eigen.dense_spectrum(A)
    wins = [eigen.window_from_spectrum(ea, Ua, s, nev) for s in shifts]
    c = partition.combine(wins, 60.0)
    return transport.transmission_spectral(c.eps, c.U, gL, gR, E), ea, Ua, c, gL, gR


def test_gradient_matches_central_differences():
    w = small_workload(4, 4, 8, 2, seed=13, amp=0.6, width=1.5)
    g = w.grid
    ab = np.array(w.absorber.as_tuple())
    shifts, nev = [-1.0, 1.0], 8
    T0, ea, Ua, c, gL, gR = _pipeline_T(g.nx, g.ny, g.nz, g.h, w.V, ab, shifts, nev, [0.0])
    E = transport.energy_grid(c.eps, 5)
    wts = np.linspace(0.5, 1.5, len(E))
    T0, ea, Ua, c, gL, gR = _pipeline_T(g.nx, g.ny, g.nz, g.h, w.V, ab, shifts, nev, E)
    in_set = np.zeros(len(ea), bool)
    for x in c.eps:
        in_set[int(np.argmin(np.abs(ea - x)))] = True
    assert in_set.sum() == len(c.eps) < g.n
    dg = gradient.absorber_param_derivs(g.nx, g.ny, g.nz, g.h, ab)
    gr = gradient.gradient_full_basis(ea, Ua, in_set, gL, gR, dg, E, wts)
    L = lambda V, a: float(wts @ _pipeline_T(g.nx, g.ny, g.nz, g.h, V, a, shifts, nev, E)[0])
    step = 1e-5
    rng = np.random.default_rng(0)
    for r in rng.choice(g.n, 6, replace=False):
        dv = np.zeros(g.n); dv[r] = step
        fd = (L(w.V + dv, ab) - L(w.V - dv, ab)) / (2 * step)
        assert abs(fd - gr["V"][r]) <= 1e-6 * max(1.0, abs(fd)), (r, fd, gr["V"][r])
    for p, ip in enumerate([0, 1, 3, 4]):
        da = np.zeros(6); da[ip] = step
        fd = (L(w.V, ab + da) - L(w.V, ab - da)) / (2 * step)
        assert abs(fd - gr["abs"][p]) <= 1e-6 * max(1.0, abs(fd)), (p, fd, gr["abs"][p])


def test_gradient_projected_matches_central_differences():
    # Tier B (set S alone, bordered sparse solves) against central
    # differences of the oracle pipeline, on the same system as above.
    w = small_workload(4, 4, 8, 2, seed=13, amp=0.6, width=1.5)
    g = w.grid
    ab = np.array(w.absorber.as_tuple())
    shifts, nev = [-1.0, 1.0], 8
    T0, ea, Ua, c, gL, gR = _pipeline_T(g.nx, g.ny, g.nz, g.h, w.V, ab, shifts, nev, [0.0])
    E = transport.energy_grid(c.eps, 5)
    wts = np.linspace(0.5, 1.5, len(E))
    As = op.assemble_sparse(g.nx, g.ny, g.nz, g.h, w.V, gL, gR)
    dg = gradient.absorber_param_derivs(g.nx, g.ny, g.nz, g.h, ab)
    gr = gradient.gradient_projected(As, c.eps, c.U, gL, gR, dg, E, wts)
    L = lambda V, a: float(wts @ _pipeline_T(g.nx, g.ny, g.nz, g.h, V, a, shifts, nev, E)[0])
    step = 1e-5
    rng = np.random.default_rng(1)
    for r in rng.choice(g.n, 6, replace=False):
        dv = np.zeros(g.n); dv[r] = step
        fd = (L(w.V + dv, ab) - L(w.V - dv, ab)) / (2 * step)
        assert abs(fd - gr["V"][r]) <= 1e-6 * max(1.0, abs(fd)), (r, fd, gr["V"][r])
    for p, ip in enumerate([0, 1, 3, 4]):
        da = np.zeros(6); da[ip] = step
        fd = (L(w.V, ab + da) - L(w.V, ab - da)) / (2 * step)
        assert abs(fd - gr["abs"][p]) <= 1e-6 * max(1.0, abs(fd)), (p, fd, gr["abs"][p])


def test_gradient_projected_equals_full_basis_on_interior_window():
    # The two tiers compute the same derivative by different routes (the
    # full eigen-expansion against sparse solves with S alone): an interior
    # window of 12 on an 8 x 8 x 12 grid, whose out-of-set part is large.
    w = small_workload(8, 8, 12, 3, seed=11)
    g = w.grid
    ab = w.absorber.as_tuple()
    gL, gR = op.gamma_fields(g.nx, g.ny, g.nz, g.h, ab)
    A = op.assemble_dense(g.nx, g.ny, g.nz, g.h, w.V, gL, gR)
    As = op.assemble_sparse(g.nx, g.ny, g.nz, g.h, w.V, gL, gR)
    ea, Ua = eigen.dense_spectrum(A)
    order = eigen.order_nearest(ea, float(ea[30].real))
    in_set = np.zeros(len(ea), bool)
    in_set[order[:12]] = True
    dg = gradient.absorber_param_derivs(g.nx, g.ny, g.nz, g.h, ab)
    E = np.linspace(ea[in_set].real.min() - 0.1, ea[in_set].real.max() + 0.1, 5)
    wts = np.random.default_rng(1).uniform(0.5, 1.5, 5)
    ref = gradient.gradient_full_basis(ea, Ua, in_set, gL, gR, dg, E, wts)
    got = gradient.gradient_projected(As, ea[in_set], Ua[:, in_set], gL, gR, dg, E, wts)
    assert np.abs(got["V"] - ref["V"]).max() <= 1e-10 * np.abs(ref["V"]).max()
    np.testing.assert_allclose(got["abs"], ref["abs"], rtol=1e-10, atol=1e-10 * np.abs(ref["abs"]).max())


def test_gradient_full_spectrum_equals_direct_adjoint():
    # With S = whole spectrum the out-of-set term vanishes and the gradient
    # of T wrt V(r) is 2 Re[(G Gamma_R G^H Gamma_L G)_rr] of the direct G.
    w = small_workload(3, 4, 6, 2, seed=2)
    A, gL, gR = _dense(w)
    ea, Ua = eigen.dense_spectrum(A)
    E = [float(ea[3].real) + 0.05]
    dg = gradient.absorber_param_derivs(3, 4, 6, 0.5, w.absorber.as_tuple())
    gr = gradient.gradient_full_basis(ea, Ua, np.ones(len(ea), bool), gL, gR, dg, E, [1.0])
    G = np.linalg.inv(E[0] * np.eye(len(ea)) - A)
    direct = 2 * np.real(np.diag(G @ np.diag(gR) @ G.conj().T @ np.diag(gL) @ G))
    np.testing.assert_allclose(gr["V"], direct, rtol=1e-8, atol=1e-12)


def test_sampled_windows_uniform_spectrum_closed_form():
    # An evenly spaced spectrum e_min + d k: every sample of 8 consecutive
    # eigenvalues measures density 1/d, the counting function is (E - e_min)/d
    # + const, and windows of n eigenvalues sit at e_min + d (n/2 + n j) up to
    # the half-spacing offset of the first sample's mean.
    d, e_min = 0.01, -1.0
    spectrum = e_min + d * np.arange(400)
    samples = [spectrum[i:i + 8] for i in range(0, 392, 40)]
    shifts = partition.sampled_windows(e_min, samples, [50, 50, 50])
    np.testing.assert_allclose(shifts, [e_min + d * (25 + 50 * j) for j in range(3)], atol=1e-12)
    # monotone and separated by n d for equal counts
    np.testing.assert_allclose(np.diff(shifts), 50 * d, atol=1e-12)


def test_semiclassical_count_tracks_exact_counts():
    # The phase-space estimate of the counting function against brute-force
    # counts of the dense spectrum, on two small systems: within 10% once 40
    # or more eigenvalues lie below E (the surface term matters: without it
    # the estimate is 40-60% high on these small boxes).
    from oracle import operator as op, eigen, partition
    from synth.workloads import workload, small_workload
    for w in (workload("c1"), small_workload(12, 10, 14, 3, seed=71)):
        g = w.grid
        gL, gR = op.gamma_fields(g.nx, g.ny, g.nz, g.h, w.absorber.as_tuple())
        ea, _ = eigen.dense_spectrum(op.assemble_dense(g.nx, g.ny, g.nz, g.h, w.V, gL, gR))
        re = np.sort(ea.real)
        shape = (g.nx, g.ny, g.nz)
        for E in np.linspace(re[40], re[min(400, len(re) - 1)], 9):
            exact = np.sum(re <= E)
            est = partition.semiclassical_count(w.V, g.h, shape, E)
            assert abs(est - exact) <= 0.10 * exact, (E, exact, est)


def test_semiclassical_windows_are_interval_midpoints():
    from oracle import partition
    from synth.workloads import workload
    w = workload("c1")
    g = w.grid
    shape = (g.nx, g.ny, g.nz)
    e_min = float(w.V.min())
    counts = [20, 30, 10]
    sh = partition.semiclassical_windows(w.V, g.h, shape, e_min, counts)
    assert all(a < b for a, b in zip(sh, sh[1:]))
    # each shift lies where the estimated count is halfway through its window
    acc = 0
    for s, c in zip(sh, counts):
        n = partition.semiclassical_count(w.V, g.h, shape, s)
        assert acc - 1e-6 <= n <= acc + c + 1e-6
        acc += c


# ---------------------------------------------------------- hole filling
def test_hole_fill_windows_worked_values():
    # Algorithm 1's repeat loop: E_S at the middle of the gap, n = 3/2 gap / Delta.
    # E_max - E_min = 8, N = 1024: Delta = 1/128; gap 0.5 -> 96 eigenpairs.
    parts = [np.array([1.0, 1.2, 1.5]), np.array([2.0, 2.3]), np.array([2.2, 2.6]), np.array([2.5, 3.0])]
    holes = [True, False, True]
    got = partition.hole_fill_windows(parts, holes, 1.0, 9.0, 1024, 200, 1e-6)
    # interface 2: gap 2.5 - 2.6 < 0 -> one eigenpair at the midpoint
    assert got == [(1.75, 96), (2.55, 1)]
    got = partition.hole_fill_windows(parts, holes, 1.0, 9.0, 1024, 50, 1e-6)
    assert got == [(1.75, 50), (2.55, 1)]
    assert partition.hole_fill_windows(parts, [False] * 3, 1.0, 9.0, 1024, 50, 1e-6) == []
    # E_min = 0.5 lies below the lowest computed value 1.0: gap 0.5 at the bottom
    got = partition.hole_fill_windows(parts, [False] * 3, 0.5, 8.5, 1024, 200, 1e-6)
    assert got == [(0.75, 96)]
    # within tau of E_min: no bottom gap
    assert partition.hole_fill_windows(parts, [False] * 3, 1.0 - 1e-9, 9.0, 1024, 200, 1e-6) == []


def test_hole_filling_closes_gaps_brute_force():
    # two windows far apart, neither reaching E_min: the loop inserts
    # partitions until no interface is flagged and E_min is reached, and the
    # combined set is then every eigenvalue of the dense spectrum up to its
    # highest real part
    w = small_workload(7, 6, 12, 3, seed=21)
    A, gL, gR = _dense(w)
    g = w.grid
    ea, Ua = eigen.dense_spectrum(A)
    nrm = op.gershgorin_norm(g.h, w.V, (gL + gR).max())
    emin = float(ea.real.min())
    emax = op.kinetic_upper_bound(g.h) + float(w.V.max())
    er = np.sort(ea.real)
    solve = lambda s, k: eigen.window_from_spectrum(ea, Ua, s, k)
    comb0 = partition.combine([solve(er[2], 6), solve(er[45], 6)], nrm)
    assert comb0.holes[0]
    comb, wins, rounds = partition.solve_with_hole_filling(solve, [(er[45], 6), (er[2], 6)], nrm, emin, emax,
                                                           g.n, 6, 10)
    assert rounds >= 2 and not comb.holes.any()
    assert [s for s, _ in wins] == sorted(s for s, _ in wins)
    lo, hi = comb.eps.real.min(), comb.eps.real.max()
    assert lo == emin
    want = np.sort_complex(ea[(ea.real >= lo) & (ea.real <= hi)])
    np.testing.assert_allclose(np.sort_complex(comb.eps), want, atol=1e-12)
    np.testing.assert_allclose(comb.U.T @ comb.U, np.eye(len(comb.eps)), atol=1e-8)


# ---------------------------------------------------------------- pins of helpers
def test_backward_error_worked_value():
    """A = diag(1, 2), u = (1, 1), theta = 3/2: r = (-1/2, 1/2), so
    ||r|| / (||A|| ||u||) = (1/sqrt 2) / (2 sqrt 2) = 1/4 with ||A|| = 2; an
    exact eigenpair gives 0."""
    A = np.diag([1.0, 2.0]).astype(complex)
    u = np.array([1.0, 1.0], dtype=complex)
    assert abs(eigen.backward_error(A, u, 1.5, 2.0) - 0.25) < 1e-15
    assert eigen.backward_error(A, np.array([0.0, 3.0j]), 2.0, 2.0) == 0.0
    # scaling u or ||A|| scales as stated
    assert abs(eigen.backward_error(A, 7.0 * u, 1.5, 4.0) - 0.125) < 1e-15


@pytest.mark.parametrize("n_r,p,want", [(10, 3, [4, 3, 3]), (400, 8, [50] * 8), (7, 7, [1] * 7),
                                        (9, 4, [3, 2, 2, 2]), (5, 1, [5]), (3, 5, [1, 1, 1, 0, 0])])
def test_equal_counts_worked_values(n_r, p, want):
    """n_r pairs dealt to p partitions as evenly as integers allow: the
    counts sum to n_r, differ by at most one, and the larger ones come
    first (worked by hand)."""
    got = partition.equal_counts(n_r, p)
    assert got == want
    assert sum(got) == n_r and max(got) - min(got) <= 1


@pytest.mark.parametrize("e_min,n_r,p,box", [(-2.65, 400, 8, (15.5, 15.5, 31.5)), (-1.0, 40, 2, (4.5, 4.5, 9.5)),
                                             (0.3, 100, 5, (10.0, 10.0, 10.0))])
def test_sample_shifts_cover_the_free_particle_region(e_min, n_r, p, box):
    """Density sampling's shifts (a reading: the paper asks for a few pairs at
    several sample points) must be max(2p, 8) evenly spaced points, each in
    the middle of its slice of [E_min, top], where `top` lies above the
    energy at which the free-particle (Weyl) count of the box reaches n_r,
    so that the samples reach the region the n_r pairs occupy."""
    s = partition.sample_shifts(e_min, n_r, p, box)
    S = max(2 * p, 8)
    assert len(s) == S
    d = np.diff(s)
    assert np.allclose(d, d[0], rtol=1e-12, atol=0) and d[0] > 0
    top = s[-1] + d[0] / 2
    assert abs((s[0] - d[0] / 2) - e_min) < 1e-12
    vol = box[0] * box[1] * box[2]
    # Weyl: N(E) = vol (2E)^(3/2) / (6 pi^2) free states below E
    e_weyl = 0.5 * (6 * math.pi ** 2 * n_r / vol) ** (2.0 / 3.0)
    assert top > e_weyl
    assert top > e_min


def test_absorber_profile_width_is_the_standard_deviation():
    """Gaussian absorbers with amplitude a and width w read as the peak and
    the standard deviation: Gamma_L(0) = a, Gamma_L(w) = a e^(-1/2)
    (e.g. 0.5 Ha and 2 bohr give 0.5 e^(-1/2) at z = 2 bohr), the half
    maximum sits at w sqrt(2 ln 2), and the mass over the half line is
    a w sqrt(pi/2).  Gamma_R is the mirror image about z_R."""
    h, nz = 0.5, 41
    zR = (nz - 1) * h
    gL, gR = op.absorber_profiles(nz, h, (0.5, 2.0, 0.0, 0.25, 3.0, zR))
    assert abs(gL[0] - 0.5) < 1e-15 and abs(gL[4] - 0.5 * math.exp(-0.5)) < 1e-15
    assert abs(gR[-1] - 0.25) < 1e-15 and abs(gR[-1 - 6] - 0.25 * math.exp(-0.5)) < 1e-15
    # fine grid: FWHM and half-line mass
    hf = 1e-3
    z = np.arange(0, 40.0, hf)
    gf, _ = op.absorber_profiles(len(z), hf, (0.5, 2.0, 0.0, 0.0, 1.0, 0.0))
    zhalf = z[np.argmin(np.abs(gf - 0.25))]
    assert abs(zhalf - 2.0 * math.sqrt(2 * math.log(2))) < 2e-3
    mass = np.trapezoid(gf, z)
    assert abs(mass - 0.5 * 2.0 * math.sqrt(math.pi / 2)) < 1e-6
    # the fields repeat the z profile over each xy plane (x fastest)
    GL, GR = op.gamma_fields(3, 2, nz, h, (0.5, 2.0, 0.0, 0.25, 3.0, zR))
    assert GL.shape == (3 * 2 * nz,) and np.all(GL[:6] == gL[0]) and np.all(GL[6:12] == gL[1])
    assert np.all(GR[-6:] == gR[-1])


def test_imaginary_bands_worked_values():
    """Two bands over Im in [-0.5, 0]: centres -1/8 and -3/8 (worked by hand),
    counts 50 -> 25 + 25 and 7 -> 4 + 3; one band keeps the window on the
    line Im = -gamma_max/2."""
    got = partition.imaginary_bands([(0.3, 50), (1.0, 7)], 0.5, 2)
    assert got == [(complex(0.3, -0.125), 25), (complex(0.3, -0.375), 25),
                   (complex(1.0, -0.125), 4), (complex(1.0, -0.375), 3)]
    assert partition.imaginary_bands([(0.3, 5)], 0.5, 1) == [(complex(0.3, -0.25), 5)]
    three = partition.imaginary_bands([(0.0, 2)], 0.6, 3)
    assert [c for _, c in three] == [1, 1, 1]
    assert np.allclose([z.imag for z, _ in three], [-0.1, -0.3, -0.5])


def test_complex_window_is_nearest_in_the_plane():
    """The window of a complex shift is the nev eigenvalues nearest it in the
    complex plane (Eq. (3) with a complex E_S), checked on a diagonal
    operator whose eigenvalues are known."""
    eps = np.array([0.0 - 0.0j, 0.1 - 0.9j, 0.2 - 0.1j, 0.5 - 1.0j, 1.0 - 0.05j])
    U = np.eye(5, dtype=complex)
    e, _ = eigen.window_from_spectrum(eps, U, complex(0.3, -0.95), 2)
    assert set(np.round(e, 12)) == {0.1 - 0.9j, 0.5 - 1.0j}
    e, _ = eigen.window_from_spectrum(eps, U, 0.3, 2)
    assert set(np.round(e, 12)) == {0.2 - 0.1j, 0.0 - 0.0j}
