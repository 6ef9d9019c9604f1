"""Transmission T(E) = Tr{G(E) Gamma_R G(E)^dagger Gamma_L} (Section 1).

Test infrastructure only (see oracle/__init__.py).

Section 1: G(E) = {E - (H - i Gamma)}^{-1}; the eigenpairs of Eq. (1) are an
intermediate that replaces the inversion.  The paper builds G from the
eigenpairs as in its TRANSEC reference, which is not reproduced in the paper;
the reading used here is the spectral sum over the computed set S of
c-normalised eigenpairs (U^T U = I for complex-symmetric A):

    G_S(E) = sum_{k in S} u_k u_k^T / (E - eps_k),

which equals (E - A)^{-1} when S is the whole spectrum.  Then

    T_S(E) = sum_{k,l} g_k conj(g_l) M^R_{kl} M^L_{kl},
    M^X = U^T Gamma_X conj(U),  g_k = 1 / (E - eps_k).

transmission_direct evaluates the definition with a dense inverse and is the
pin for the spectral form at full spectrum on small grids.
"""
from __future__ import annotations

import numpy as np


def energy_grid(eps: np.ndarray, n_e: int) -> np.ndarray:
    """n_E uniform energies over [min Re eps, max Re eps], ends included
    (reading: the synthetic systems have no Fermi level)."""
    re = np.asarray(eps).real
    if n_e == 1:
        return np.array([0.5 * (re.min() + re.max())])
    return np.linspace(re.min(), re.max(), n_e)


def gamma_gram(U: np.ndarray, gamma: np.ndarray) -> np.ndarray:
    """M = U^T diag(gamma) conj(U): Hermitian positive semidefinite."""
    return U.T @ (gamma[:, None] * U.conj())


def transmission_spectral(eps: np.ndarray, U: np.ndarray, gL: np.ndarray,
                          gR: np.ndarray, energies: np.ndarray) -> np.ndarray:
    MR = gamma_gram(U, gR)
    ML = gamma_gram(U, gL)
    W = MR * ML
    T = np.empty(len(energies))
    for e, E in enumerate(energies):
        g = 1.0 / (E - eps)
        T[e] = float(np.real(g @ W @ g.conj()))
    return T


def transmission_direct(A_dense: np.ndarray, gL: np.ndarray, gR: np.ndarray,
                        energies: np.ndarray) -> np.ndarray:
    N = A_dense.shape[0]
    T = np.empty(len(energies))
    for e, E in enumerate(energies):
        G = np.linalg.inv(E * np.eye(N) - A_dense)
        T[e] = float(np.real(np.trace(G @ (gR[:, None] * G.conj().T) @ np.diag(gL))))
    return T
