"""Per-window eigenpairs of A nearest a real shift (Eq. (3)).

Test infrastructure only (see oracle/__init__.py).

Section 2: each partition j solves (A - E_{S,j}) U = (eps - E_{S,j}) U for the
n_{r,j} eigenvalues closest to the shift; Section 2.1 obtains them with
ARPACK's 'SM' (smallest magnitude) option on the shifted operator, without
inversion.  The eigenvectors are bi-orthogonal under the unconjugated product
(Section 1), so they are scaled to u^T u = 1.

Because the window result has a plain definition (the n eigenpairs with
smallest |eps - sigma|), this module computes that definition:
  * tier A (small N): dense eigendecomposition of the assembled A;
  * tier B (large N): ARPACK 'SM' on A - sigma through scipy, i.e. the
    paper's own library call, with a guard band of extra eigenpairs so the
    n nearest are chosen exactly, then a c-Rayleigh-quotient polish.

Readings: distance is the complex modulus |eps - sigma|; ties are broken by
(Re eps, Im eps) ascending; c-normalisation uses the principal square root.
"""
from __future__ import annotations

from typing import Tuple

import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as sla


def c_normalize(U: np.ndarray) -> np.ndarray:
    """Scale each column to u^T u = 1 (unconjugated product, Section 1)."""
    U = np.array(U, dtype=np.complex128, copy=True)
    if U.ndim == 1:
        return U / np.sqrt(U @ U)
    return U / np.sqrt(np.sum(U * U, axis=0))[None, :]


def c_rayleigh(A, u: np.ndarray) -> complex:
    """u^T A u / u^T u: the Rayleigh quotient under the unconjugated product.

    For complex-symmetric A its error is quadratic in the eigenvector error."""
    Au = A @ u
    return complex((u @ Au) / (u @ u))


def backward_error(A, u: np.ndarray, theta: complex, norm_a: float) -> float:
    """||A u - theta u||_2 / (||A|| ||u||_2)."""
    r = A @ u - theta * u
    return float(np.linalg.norm(r) / (norm_a * np.linalg.norm(u)))


def order_nearest(eps: np.ndarray, sigma: float) -> np.ndarray:
    """Indices of eps by increasing |eps - sigma|, ties by (Re, Im)."""
    eps = np.asarray(eps)
    return np.lexsort((eps.imag, eps.real, np.abs(eps - sigma)))


def order_real(eps: np.ndarray) -> np.ndarray:
    """Ordering by real part (the paper's only ordering, Section 2 footnote)."""
    eps = np.asarray(eps)
    return np.lexsort((eps.imag, eps.real))


def dense_spectrum(A_dense: np.ndarray) -> Tuple[np.ndarray, np.ndarray]:
    """All eigenpairs of A (tier A), c-normalised, in ascending real part."""
    eps, U = np.linalg.eig(A_dense)
    o = order_real(eps)
    return eps[o], c_normalize(U[:, o])


def window_dense(A_dense: np.ndarray, sigma: float, nev: int):
    """The nev eigenpairs nearest sigma, from the full spectrum (tier A)."""
    eps, U = dense_spectrum(A_dense)
    idx = order_nearest(eps, sigma)[:nev]
    idx = idx[order_real(eps[idx])]
    return eps[idx], U[:, idx]


def window_from_spectrum(eps: np.ndarray, U: np.ndarray, sigma: float, nev: int):
    idx = order_nearest(eps, sigma)[:nev]
    idx = idx[order_real(eps[idx])]
    return eps[idx], U[:, idx]


def window_arpack(A_sparse: sp.spmatrix, sigma: float, nev: int, guard: int = 8,
                  ncv: int = 0, tol: float = 1e-13, maxiter: int = 200000):
    """The nev eigenpairs nearest sigma via ARPACK 'SM' on A - sigma (tier B).

    Section 2.1: the shift moves the window to the origin and the 'SM' option
    selects the eigenvalues of smallest magnitude of the shifted operator.
    nev + guard pairs are requested so that the nev nearest are exact; each
    returned pair is c-normalised and its eigenvalue replaced by the
    c-Rayleigh quotient (quadratically accurate)."""
    N = A_sparse.shape[0]
    k = min(nev + guard, N - 2)
    ncv = ncv or min(N - 1, max(2 * k + 1, k + 40))
    B = (A_sparse - sigma * sp.identity(N, format="csr")).tocsr()
    w, U = sla.eigs(B, k=k, which="SM", ncv=ncv, tol=tol, maxiter=maxiter)
    U = c_normalize(U)
    AU = A_sparse @ U
    eps = np.sum(U * AU, axis=0) / np.sum(U * U, axis=0)
    idx = order_nearest(eps, sigma)[:nev]
    idx = idx[order_real(eps[idx])]
    return eps[idx], U[:, idx]


def lowest_real(A_sparse: sp.spmatrix, k: int, tol: float = 1e-13) -> np.ndarray:
    """The k eigenvalues of smallest real part (Section 2.2: the exterior end of
    the spectrum where the partitioned interval starts), by ARPACK 'SR' with
    eigenvectors; each eigenvalue is replaced by its c-Rayleigh quotient and the
    result is sorted by real part."""
    N = A_sparse.shape[0]
    kk = min(k + 4, N - 2)
    w, U = sla.eigs(A_sparse, k=kk, which="SR", tol=tol, ncv=min(N - 1, max(40, 3 * kk)),
                    maxiter=200000)
    U = c_normalize(U)
    eps = np.sum(U * (A_sparse @ U), axis=0) / np.sum(U * U, axis=0)
    return eps[order_real(eps)][:k]



def lowest_real_pairs(A_sparse: sp.spmatrix, k: int, guard: int = 24, ncv: int = 0, tol: float = 1e-12):
    """The k eigenpairs of smallest real part (the exterior end of the
    spectrum, Section 2.2), by ARPACK 'SR' on k + guard pairs; each pair is
    c-normalised, its eigenvalue replaced by the c-Rayleigh quotient, and the
    result sorted by real part.  The guard pairs are computed and dropped,
    so that the k returned are the lowest (an eigenvalue of the same real
    part can only be missed inside the guard band).
    Returns (eps, U, e_trust) with e_trust the real part below which the set
    holds every eigenvalue: the largest real part among the returned pairs."""
    N = A_sparse.shape[0]
    kk = min(k + guard, N - 2)
    ncv = ncv or min(N - 1, 2 * kk + 40)
    w, U = sla.eigs(A_sparse, k=kk, which="SR", tol=tol, ncv=ncv, maxiter=200000)
    U = c_normalize(U)
    eps = np.sum(U * (A_sparse @ U), axis=0) / np.sum(U * U, axis=0)
    o = order_real(eps)[:k]
    eps, U = eps[o], U[:, o]
    return eps, U, float(eps.real.max())
