"""Pins for oracle.operator and the dense eigen-route (CPU only).

Each check ties the oracle to something other than itself: exact moment
conditions of the FD weights, a published weight table, an independent
Kronecker-sum assembly, the plane-wave symbol, closed-form spectra of the
discrete Laplacian, and the trace identity.
"""
import json
import os
from fractions import Fraction

import numpy as np
import pytest

from oracle import operator as op
from oracle import eigen
from synth.workloads import Grid, small_workload

GOLD = os.path.join(os.path.dirname(__file__), "golden")


@pytest.mark.parametrize("R", [1, 2, 3, 4, 5, 6])
def test_fd_moments_exact(R):
    # sum_{m=-R..R} c_|m| m^(2q) = 2 for q = 1 and 0 for q = 0, 2..R:
    # the weights reproduce d^2/dx^2 exactly on polynomials of degree 2R+1.
    c = op.fd_coefficients(R)
    for q in range(0, R + 1):
        s = c[0] * (1 if q == 0 else 0) + 2 * sum(c[m] * Fraction(m) ** (2 * q) for m in range(1, R + 1))
        assert s == (2 if q == 1 else 0), (R, q, s)


def test_fd_weights_published_table():
    table = json.load(open(os.path.join(GOLD, "fd_weights.json")))["weights"]
    for R, ws in table.items():
        assert op.fd_coefficients(int(R)) == [Fraction(w) for w in ws]


def _random_fields(nx, ny, nz, seed):
    rng = np.random.default_rng(seed)
    V = rng.uniform(-3, 1, nx * ny * nz)
    ab = (0.4, 1.5, 0.0, 0.3, 1.2, (nz - 1) * 0.5)
    gL, gR = op.gamma_fields(nx, ny, nz, 0.5, ab)
    return V, gL, gR


@pytest.mark.parametrize("shape", [(7, 5, 9), (13, 14, 15), (3, 4, 20)])
@pytest.mark.parametrize("R", [1, 6])
def test_matvec_matches_kronecker_assembly(shape, R):
    nx, ny, nz = shape
    V, gL, gR = _random_fields(nx, ny, nz, 1)
    A = op.assemble_sparse(nx, ny, nz, 0.5, V, gL, gR, R)
    rng = np.random.default_rng(2)
    X = rng.standard_normal((nx * ny * nz, 3)) + 1j * rng.standard_normal((nx * ny * nz, 3))
    Y = op.apply_operator(nx, ny, nz, 0.5, V, gL, gR, X, R)
    np.testing.assert_allclose(Y, A @ X, rtol=0, atol=1e-12 * np.abs(A @ X).max())
    # complex symmetric, not Hermitian (Section 1)
    Ad = A.toarray()
    assert np.abs(Ad - Ad.T).max() == 0.0
    assert np.abs(Ad - Ad.conj().T).max() > 0.1


def test_plane_wave_symbol_interior():
    # Far (>= R points) from every wall the truncated stencil acts on
    # exp(i theta . r) as the infinite one: eigenvalue (1/2h^2) sum s(theta_a).
    nx = ny = nz = 16
    h = 0.37
    th = np.array([0.3, 1.1, 2.9])
    i, j, k = np.meshgrid(np.arange(nx), np.arange(ny), np.arange(nz), indexing="xy")
    # build x fastest: index = i + nx (j + ny k)
    kk, jj, ii = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    x = np.exp(1j * (th[0] * ii + th[1] * jj + th[2] * kk)).reshape(-1)
    zero = np.zeros(nx * ny * nz)
    y = op.apply_operator(nx, ny, nz, h, zero, zero, zero, x, 6)
    lam = sum(op.symbol(t) for t in th) / (2 * h * h)
    inner = (ii >= 6) & (ii < nx - 6) & (jj >= 6) & (jj < ny - 6) & (kk >= 6) & (kk < nz - 6)
    inner = inner.reshape(-1)
    np.testing.assert_allclose(y[inner], lam * x[inner], atol=1e-11)
    # symbol approximates theta^2 (12th order)
    assert abs(op.symbol(0.1) - 0.01) < 1e-14


def test_closed_form_spectrum_radius1():
    # R = 1 with V = Gamma = 0: eigenvalues are sums of (1 - cos(pi k/(n+1)))/h^2.
    nx, ny, nz, h = 4, 5, 6, 0.5
    z = np.zeros(nx * ny * nz)
    A = op.assemble_dense(nx, ny, nz, h, z, z, z, 1)
    eps, U = eigen.dense_spectrum(A)
    one = lambda n: (1 - np.cos(np.pi * np.arange(1, n + 1) / (n + 1))) / h ** 2
    ref = np.sort((one(nx)[:, None, None] + one(ny)[None, :, None] + one(nz)[None, None, :]).ravel())
    np.testing.assert_allclose(np.sort(eps.real), ref, atol=1e-12)
    assert np.abs(eps.imag).max() < 1e-12


def test_closed_form_spectrum_radius6_separable():
    # R = 6, V = Gamma = 0: Kronecker-sum spectrum from three 1-D
    # symmetric eigenproblems (LAPACK eigvalsh) equals the 3-D dense spectrum.
    nx, ny, nz, h = 5, 6, 8, 0.5
    z = np.zeros(nx * ny * nz)
    A = op.assemble_dense(nx, ny, nz, h, z, z, z, 6)
    eps = np.sort(np.linalg.eigvals(A).real)
    l = [np.linalg.eigvalsh(op.laplacian_1d(n, h, 6)) for n in (nx, ny, nz)]
    ref = np.sort((l[0][:, None, None] + l[1][None, :, None] + l[2][None, None, :]).ravel())
    np.testing.assert_allclose(eps, ref, atol=1e-11)
    # every 1-D eigenvalue lies below the symbol bound
    assert max(x.max() for x in l) <= op.kinetic_upper_bound(h) / 3 + 1e-12


def test_trace_identity_and_im_bound():
    w = small_workload(6, 5, 8, 3, seed=11, amp=0.7, width=1.3)
    g = w.grid
    gL, gR = op.gamma_fields(g.nx, g.ny, g.nz, g.h, w.absorber.as_tuple())
    A = op.assemble_dense(g.nx, g.ny, g.nz, g.h, w.V, gL, gR)
    eps, U = eigen.dense_spectrum(A)
    c0 = float(op.fd_coefficients(6)[0])
    tr = g.n * (-3 * c0 / (2 * g.h ** 2)) + w.V.sum() - 1j * (gL + gR).sum()
    assert abs(eps.sum() - tr) < 1e-9 * abs(tr)
    # Eq. (5): 0 <= -Im eps <= max Gamma (exact: Im eps = -u^H Gamma u/u^H u)
    gmax = (gL + gR).max()
    assert eps.imag.max() <= 1e-12 and (-eps.imag).max() <= gmax + 1e-12
    # bi-orthogonality U^T U = I (Section 1)
    np.testing.assert_allclose(U.T @ U, np.eye(g.n), atol=1e-9)
    # Re eps below the exact bound used for E_max
    assert eps.real.max() <= op.kinetic_upper_bound(g.h) + w.V.max() + 1e-9


def test_eq5_first_order_slope():
    # Scaling Gamma by alpha: Im eps_k = -alpha <u_k^KS|Gamma|u_k^KS> + O(alpha^2)
    w = small_workload(5, 5, 8, 2, seed=5)
    g = w.grid
    gL, gR = op.gamma_fields(g.nx, g.ny, g.nz, g.h, w.absorber.as_tuple())
    z = np.zeros(g.n)
    H = op.assemble_dense(g.nx, g.ny, g.nz, g.h, w.V, z, z)
    ks, U0 = np.linalg.eigh(H.real)
    expect = np.einsum("rk,r,rk->k", U0, gL + gR, U0)[:5]
    for alpha in (1e-4, 2e-4):
        A = op.assemble_dense(g.nx, g.ny, g.nz, g.h, w.V, alpha * gL, alpha * gR)
        eps, _ = eigen.dense_spectrum(A)
        np.testing.assert_allclose(-eps.imag[:5] / alpha, expect, rtol=1e-3)
        np.testing.assert_allclose(eps.real[:5], ks[:5], atol=1e-6)


def test_gershgorin_bound_dominates():
    w = small_workload(6, 6, 10, 3, seed=3)
    g = w.grid
    gL, gR = op.gamma_fields(g.nx, g.ny, g.nz, g.h, w.absorber.as_tuple())
    A = op.assemble_dense(g.nx, g.ny, g.nz, g.h, w.V, gL, gR)
    nrm = op.gershgorin_norm(g.h, w.V, (gL + gR).max())
    assert np.linalg.norm(A, 2) <= nrm
    # h = 0.5: kinetic part of the bound is 42.44 Ha
    assert abs(op.kinetic_upper_bound(0.5) - 42.4374) < 1e-3
