"""Exact derivative of L = sum_e w_e T_S(E_e) with respect to the potential
V(r) and the four absorber parameters (a_L, w_L, a_R, w_R).

Test infrastructure only (see oracle/__init__.py).

The paper never differentiates T(E); this is the derivative of the quantity
the pipeline computes (T_S of transport.py, energies held fixed).  With
dA = diag(dV) - i diag(dGamma), c-normalised eigenpairs (u^T u = 1) and
g_k = 1/(E - eps_k):

  d eps_k = u_k^T dA u_k                       (first order, cf. Eq. (5))
  dG_S    = G_S dA G_S + sum_{k in S} g_k (w_k u_k^T + u_k w_k^T),
  w_k     = Q (eps_k - A)^{-1} Q dA u_k,   Q = I - U_S U_S^T,

  dT = 2 Re Tr{dG_S Gamma_R G_S^H Gamma_L}
       + Tr{G_S dGamma_R G_S^H Gamma_L} + Tr{G_S Gamma_R G_S^H dGamma_L}.

In adjoint form the out-of-set term is 2 Re sum_k lambda_k^T dA u_k with
lambda_k = Q (eps_k - A)^{-1} Q s_k and
s_k = sum_e w_e g_k(E_e) (Gamma_R conj(G_S) Gamma_L + Gamma_L conj(G_S) Gamma_R) u_k.
gradient_full_basis (tier A) evaluates the projected solve in the full
eigenbasis: lambda_k = sum_{l not in S} u_l (u_l^T s_k) / (eps_k - eps_l).
gradient_projected (tier B) needs only S: the in-set terms are contractions
through n x n Grams, and each lambda_k is a direct sparse solve of the
bordered system  [eps_k - A, -U_S; U_S^T, 0] [lambda; mu] = [Q s_k; 0],
whose solution is exactly lambda_k = Q (eps_k - A)^{-1} Q s_k (A commutes
with Q because A U_S = U_S diag(eps_S) and U_S^T U_S = I; the system is
nonsingular when eps_k is not also an eigenvalue outside S).
"""
from __future__ import annotations

from typing import Dict, Sequence

import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla


def absorber_param_derivs(nx, ny, nz, h, absorber):
    """d Gamma_X / d(a_X, w_X) as length-N diagonals, in the order
    (a_L, w_L, a_R, w_R); each entry is (side, field)."""
    aL, wL, zL, aR, wR, zR = absorber
    z = np.arange(nz) * h
    eL = np.exp(-((z - zL) ** 2) / (2 * wL * wL))
    eR = np.exp(-((z - zR) ** 2) / (2 * wR * wR))
    rep = nx * ny
    return [
        ("L", np.repeat(eL, rep)),
        ("L", np.repeat(aL * eL * (z - zL) ** 2 / wL ** 3, rep)),
        ("R", np.repeat(eR, rep)),
        ("R", np.repeat(aR * eR * (z - zR) ** 2 / wR ** 3, rep)),
    ]


def gradient_full_basis(eps_all: np.ndarray, U_all: np.ndarray, in_set: np.ndarray,
                        gL: np.ndarray, gR: np.ndarray, dgamma, energies: Sequence[float],
                        weights: Sequence[float]) -> Dict[str, np.ndarray]:
    """Gradient of sum_e weights[e] T_S(E_e) (tier A: full eigenbasis known).

    eps_all, U_all: every eigenpair of A, c-normalised; in_set: bool mask of S.
    dgamma: absorber_param_derivs(...).  Returns {'V': (N,), 'abs': (4,)}.
    """
    US = U_all[:, in_set]
    eS = eps_all[in_set]
    Uo = U_all[:, ~in_set]
    eo = eps_all[~in_set]
    N = U_all.shape[0]
    dV = np.zeros(N)
    dabs = np.zeros(4)
    n_s = US.shape[1]
    S = np.zeros((N, n_s), dtype=np.complex128)   # s_k columns
    for E, wgt in zip(energies, weights):
        g = 1.0 / (E - eS)
        G = (US * g[None, :]) @ US.T
        M = gR[:, None] * G.conj().T * gL[None, :]          # Gamma_R G^H Gamma_L
        GMG = G @ M @ G
        diag_in = np.diag(GMG)                               # (G M G)_rr
        # in-set part through dA: d/dV(r) of 2 Re Tr{G dA G M}
        dV += wgt * 2.0 * np.real(diag_in)
        # absorber: dA = -i diag(dGamma)
        for p, (side, d) in enumerate(dgamma):
            dabs[p] += wgt * 2.0 * np.real(np.sum(-1j * d * diag_in))
            # explicit Gamma dependence of the trace
            if side == "R":
                dabs[p] += wgt * np.real(np.trace((G * d[None, :]) @ G.conj().T * gL[None, :]))
            else:
                dabs[p] += wgt * np.real(np.trace((G * gR[None, :]) @ G.conj().T * d[None, :]))
        Msym = M + M.T
        S += wgt * (Msym @ US) * g[None, :]
    # out-of-set part: lambda_k = sum_{l not in S} u_l (u_l^T s_k)/(eps_k - eps_l)
    coef = (Uo.T @ S) / (eS[None, :] - eo[:, None])
    Lam = Uo @ coef
    prod = Lam * US                                          # lambda_k(r) u_k(r)
    dV += 2.0 * np.real(prod.sum(axis=1))
    for p, (side, d) in enumerate(dgamma):
        dabs[p] += 2.0 * np.real(np.sum(-1j * d[:, None] * prod))
    return {"V": dV, "abs": dabs}


def gradient_projected(A_sparse, eps_S: np.ndarray, U_S: np.ndarray, gL: np.ndarray, gR: np.ndarray,
                       dgamma, energies: Sequence[float], weights: Sequence[float]) -> Dict[str, np.ndarray]:
    """Gradient of sum_e weights[e] T_S(E_e) from the set S alone (tier B).

    A_sparse: the operator (operator.assemble_sparse); eps_S, U_S: the pairs
    of S, c-normalised (U_S^T U_S = I).  Same result as gradient_full_basis.
    Returns {'V': (N,), 'abs': (4,)}.
    """
    N, n = U_S.shape
    Uc = U_S.conj()
    MR = U_S.T @ (gR[:, None] * Uc)                         # U^T Gamma_R conj(U)
    ML = U_S.T @ (gL[:, None] * Uc)
    Pd = [U_S.T @ (d[:, None] * Uc) for _, d in dgamma]
    dV = np.zeros(N)
    dabs = np.zeros(4)
    S = np.zeros((N, n), dtype=np.complex128)                # s_k columns
    for E, wgt in zip(energies, weights):
        g = 1.0 / (E - eps_S)
        gc = g.conj()
        # (G M G)_rr with G = U diag(g) U^T, M = Gamma_R conj(G) Gamma_L:
        # U^T M U = MR diag(conj g) conj(ML)
        X = (MR * gc[None, :]) @ ML.conj()
        Y = g[:, None] * X * g[None, :]
        diag_in = np.sum((U_S @ Y) * U_S, axis=1)
        dV += wgt * 2.0 * np.real(diag_in)
        for p, (side, d) in enumerate(dgamma):
            dabs[p] += wgt * 2.0 * np.real(np.sum(-1j * d * diag_in))
            # explicit Gamma dependence: Tr{G dGamma_R G^H Gamma_L} or
            # Tr{G Gamma_R G^H dGamma_L}, each a trace of n x n products
            if side == "R":
                dabs[p] += wgt * np.real(np.sum((g[:, None] * Pd[p] * gc[None, :]) * ML.conj().T))
            else:
                dabs[p] += wgt * np.real(np.sum((g[:, None] * MR * gc[None, :]) * Pd[p].conj().T))
        # (M + M^T) U, M U = Gamma_R conj(U) diag(conj g) conj(ML),
        # M^T U = Gamma_L conj(U) diag(conj g) conj(MR)
        MU = gR[:, None] * (Uc @ (gc[:, None] * ML.conj()))
        MtU = gL[:, None] * (Uc @ (gc[:, None] * MR.conj()))
        S += wgt * (MU + MtU) * g[None, :]
    # out-of-set part: one bordered sparse solve per pair of S
    A = sp.csr_matrix(A_sparse)
    I = sp.identity(N, dtype=np.complex128, format="csr")
    B = sp.csr_matrix(-U_S)
    Bt = sp.csr_matrix(U_S.T)
    Lam = np.empty((N, n), dtype=np.complex128)
    for k in range(n):
        K = sp.bmat([[eps_S[k] * I - A, B], [Bt, None]], format="csc")
        rhs = np.concatenate([S[:, k] - U_S @ (U_S.T @ S[:, k]), np.zeros(n, dtype=np.complex128)])
        Lam[:, k] = spla.splu(K).solve(rhs)[:N]
    prod = Lam * U_S
    dV += 2.0 * np.real(prod.sum(axis=1))
    for p, (side, d) in enumerate(dgamma):
        dabs[p] += 2.0 * np.real(np.sum(-1j * d[:, None] * prod))
    return {"V": dV, "abs": dabs}
