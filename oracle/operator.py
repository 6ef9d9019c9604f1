"""The real-space operator of Eq. (1): A = H - i Gamma, Gamma = Gamma_L + Gamma_R.

Test infrastructure only (see oracle/__init__.py).

Section 1 of the paper: H is a real-symmetric Kohn-Sham Hamiltonian on a
uniform real-space grid of spacing h, never stored, applied as a
matrix-vector product formula (finite differences); -i Gamma is a sum of two
imaginary, diagonal, Gaussian absorbing potentials at the two ends of the cell,
so A is complex symmetric.

Readings where the paper is silent (the synthetic stand-in for H_KS):
  * H = -1/2 Laplacian + V(r), the Laplacian by the central finite difference
    of order 2R (R = 6 by default) with zero values outside the box;
  * grid point (i, j, k) sits at (i h, j h, k h), linear index i + nx (j + ny k);
  * Gamma_X(z) = a_X exp(-(z - z_X)^2 / (2 w_X^2)), depending on z only
    (width = standard deviation, amplitude = peak value).
"""
from __future__ import annotations

from fractions import Fraction
from math import factorial
from typing import List, Sequence, Tuple

import numpy as np
import scipy.sparse as sp


def fd_coefficients(radius: int = 6) -> List[Fraction]:
    """Exact central-difference weights c_0..c_R for d^2/dx^2 of order 2R.

    c_m = 2 (-1)^(m+1) (R!)^2 / (m^2 (R-m)! (R+m)!) for m >= 1 and
    c_0 = -2 sum_m c_m, so that sum_{m=-R..R} c_|m| f(x + m h) / h^2
    approximates f''(x) with error O(h^(2R)).
    """
    if not 1 <= radius <= 6:
        raise ValueError("radius must be in 1..6")
    R = radius
    c = [Fraction(0)] * (R + 1)
    for m in range(1, R + 1):
        c[m] = Fraction(2 * (-1) ** (m + 1) * factorial(R) ** 2,
                        m * m * factorial(R - m) * factorial(R + m))
    c[0] = -2 * sum(c[1:])
    return c


def fd_coefficients_f64(radius: int = 6) -> np.ndarray:
    return np.array([float(x) for x in fd_coefficients(radius)])


def absorber_profiles(nz: int, h: float, absorber: Sequence[float]) -> Tuple[np.ndarray, np.ndarray]:
    """Gamma_L(z), Gamma_R(z) on the nz planes (Section 1: Gaussian absorbers)."""
    aL, wL, zL, aR, wR, zR = absorber
    z = np.arange(nz) * h
    gL = aL * np.exp(-((z - zL) ** 2) / (2.0 * wL * wL))
    gR = aR * np.exp(-((z - zR) ** 2) / (2.0 * wR * wR))
    return gL, gR


def gamma_fields(nx: int, ny: int, nz: int, h: float, absorber) -> Tuple[np.ndarray, np.ndarray]:
    """Gamma_L and Gamma_R as length-N diagonals (x fastest)."""
    gL, gR = absorber_profiles(nz, h, absorber)
    rep = nx * ny
    return np.repeat(gL, rep), np.repeat(gR, rep)


def apply_operator(nx, ny, nz, h, V, gL, gR, x, radius=6):
    """y = A x by the matrix-vector product formula (Section 1).

    x may be (N,) or (N, B).  Each axis contributes
    -(1/(2h^2)) sum_{m=-R..R} c_|m| x(r + m e_axis), with x = 0 outside the
    box; the diagonal adds V(r) - i (Gamma_L + Gamma_R)(r).
    """
    c = fd_coefficients_f64(radius)
    x = np.asarray(x)
    single = x.ndim == 1
    X = x.reshape(nz, ny, nx, -1).astype(np.complex128)
    scale = -1.0 / (2.0 * h * h)
    # the three axes share the centre tap, so the diagonal is 3 c_0
    Y = scale * 3.0 * c[0] * X
    for m in range(1, radius + 1):
        cm = scale * c[m]
        # x axis (last spatial axis of the (z, y, x) array)
        Y[:, :, m:, :] += cm * X[:, :, :-m, :]
        Y[:, :, :-m, :] += cm * X[:, :, m:, :]
        # y axis
        Y[:, m:, :, :] += cm * X[:, :-m, :, :]
        Y[:, :-m, :, :] += cm * X[:, m:, :, :]
        # z axis
        Y[m:, :, :, :] += cm * X[:-m, :, :, :]
        Y[:-m, :, :, :] += cm * X[m:, :, :, :]
    diag = (np.asarray(V, dtype=np.float64) - 1j * (gL + gR)).reshape(nz, ny, nx, 1)
    Y += diag * X
    Y = Y.reshape(nx * ny * nz, -1)
    return Y[:, 0] if single else Y


def laplacian_1d(n: int, h: float, radius: int = 6) -> np.ndarray:
    """Dense 1-D kinetic matrix -(1/(2h^2)) D2 with zero Dirichlet truncation."""
    c = fd_coefficients_f64(radius)
    T = np.zeros((n, n))
    for i in range(n):
        for m in range(-radius, radius + 1):
            j = i + m
            if 0 <= j < n:
                T[i, j] = c[abs(m)]
    return -T / (2.0 * h * h)


def assemble_sparse(nx, ny, nz, h, V, gL, gR, radius=6) -> sp.csr_matrix:
    """A as a sparse matrix, built as the Kronecker sum of the 1-D kinetic
    matrices plus the diagonal (an independent construction from
    apply_operator, used to cross-check it)."""
    Tx = sp.csr_matrix(laplacian_1d(nx, h, radius))
    Ty = sp.csr_matrix(laplacian_1d(ny, h, radius))
    Tz = sp.csr_matrix(laplacian_1d(nz, h, radius))
    Ix, Iy, Iz = sp.identity(nx), sp.identity(ny), sp.identity(nz)
    K = (sp.kron(sp.kron(Iz, Iy), Tx) + sp.kron(sp.kron(Iz, Ty), Ix)
         + sp.kron(sp.kron(Tz, Iy), Ix))
    D = sp.diags(np.asarray(V, dtype=np.float64) - 1j * (gL + gR))
    return (K + D).tocsr().astype(np.complex128)


def assemble_dense(nx, ny, nz, h, V, gL, gR, radius=6) -> np.ndarray:
    return assemble_sparse(nx, ny, nz, h, V, gL, gR, radius).toarray()


def symbol(theta, radius=6) -> np.ndarray:
    """s(theta) = -(c_0 + 2 sum_m c_m cos(m theta)): the 1-D stencil's Fourier
    symbol in units of 1/h^2 (the eigenvalue of -D2 on a plane wave)."""
    c = fd_coefficients_f64(radius)
    theta = np.asarray(theta, dtype=np.float64)
    s = c[0] + 2.0 * sum(c[m] * np.cos(m * theta) for m in range(1, radius + 1))
    return -s


def kinetic_upper_bound(h: float, radius: int = 6) -> float:
    """Upper bound on the eigenvalues of the 3-D kinetic part: 3 max s / (2h^2).

    The truncated (zero-Dirichlet) 1-D matrix is a principal section of the
    infinite Toeplitz operator, so its eigenvalues lie inside the range of
    the symbol."""
    th = np.linspace(0.0, np.pi, 20001)
    return 3.0 * float(symbol(th, radius).max()) / (2.0 * h * h)


def gershgorin_norm(h: float, V, gamma_max: float, radius: int = 6) -> float:
    """||A||_G: row-sum bound, used to scale the backward error.

    Every row of the kinetic part has absolute row sum at most
    3 (|c_0| + 2 sum |c_m|) / (2 h^2); add max |V| and max Gamma."""
    c = fd_coefficients_f64(radius)
    kin = 3.0 * (abs(c[0]) + 2.0 * np.abs(c[1:]).sum()) / (2.0 * h * h)
    return float(kin + np.max(np.abs(V)) + gamma_max)
