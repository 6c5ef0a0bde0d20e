"""Streamed density-fitting FP64 oracle (test infrastructure only; see the package docstring).

The same quantities as ``oracle.pnof``, rewritten for (mn|ls) = sum_P B_P B_P so that no
per-orbital AO matrix is materialised, and B is visited one row-block of P at a time:

  b_P    = C_A^T B_P C_A                 (NO-basis three-index integrals)
  K_pq   = sum_P b_P[p,q]^2              (= (pq|pq), Eq. JKpq)
  D_Pp   = b_P[p,p];  J = D^T D          (= (pp|qq), Eq. JKpq)
  Y      = n o (H C_A) + sum_P (B_P C_A) (b_P o beta + diag(D_P alpha))
           which is F^q c_q of Eq. lowdin/4 written with J^r c_q = sum_P B_P c_q D_Pr and
           K^r c_q = sum_P (B_P c_r) b_P[r,q]
  lambda = C^T Y                         (Eq. lag)

B can be an array of shape (naux, nbf, nbf) or a callable ``chunk(p0, p1)`` returning those
rows (so 55 GB of float64 never has to exist at once).
"""
from __future__ import annotations

import math

import numpy as np

from . import pnof


def _chunks(B, naux, pchunk):
    for p0 in range(0, naux, pchunk):
        p1 = min(naux, p0 + pchunk)
        yield p0, p1, (B(p0, p1) if callable(B) else B[p0:p1])


def jk(C, B, nact: int, naux: int | None = None, pchunk: int = 64):
    """J, K (nact x nact) and D (naux x nact) by one pass over B."""
    naux = B.shape[0] if naux is None else naux
    CA = C[:, :nact]
    K = np.zeros((nact, nact))
    D = np.zeros((naux, nact))
    for p0, p1, Bc in _chunks(B, naux, pchunk):
        X = Bc @ CA                                    # (P, nbf, nact)
        b = CA.T @ X                                   # (P, nact, nact)
        K += (b * b).sum(axis=0)
        D[p0:p1] = np.diagonal(b, axis1=1, axis2=2)
    return D.T @ D, K, D


def lagrangian(C, n, H, B, npairs: int, ncwo: int, functional: int = pnof.PNOF7,
               naux: int | None = None, pchunk: int = 64, nsingle: int = 0):
    """E, lambda (nbf x nbf), Y (nbf x nact), J, K, dE/dn in one pass over B.

    Returns a dict with keys E, lam, Y, J, K, Hpp, dEdn, dEdC.
    """
    naux = B.shape[0] if naux is None else naux
    nbf = C.shape[0]
    nact = npairs * (ncwo + 1) + nsingle
    n = np.asarray(n, dtype=np.float64)[:nact]
    CA = C[:, :nact]
    alpha, beta = pnof.coefficients(n, npairs, ncwo, functional, nsingle)
    HC = H @ CA
    Hpp = np.einsum("mp,mp->p", CA, HC)
    Y = HC * n[None, :]
    K = np.zeros((nact, nact))
    D = np.zeros((naux, nact))
    for p0, p1, Bc in _chunks(B, naux, pchunk):
        X = Bc @ CA                                    # (P, nbf, nact)
        b = CA.T @ X                                   # (P, nact, nact)
        K += (b * b).sum(axis=0)
        Dc = np.diagonal(b, axis1=1, axis2=2).copy()
        D[p0:p1] = Dc
        d = Dc @ alpha                                 # (P, nact): sum_r alpha_qr D_Pr
        W = b * beta[None, :, :]
        idx = np.arange(nact)
        W[:, idx, idx] += d
        for k in range(X.shape[0]):
            Y += X[k] @ W[k]
    J = D.T @ D
    E = math.fsum(np.concatenate([2.0 * n * Hpp, (alpha * J).ravel(), (beta * K).ravel()]))
    lam = np.zeros((nbf, nbf))
    lam[:, :nact] = C.T @ Y
    dEdC = np.zeros_like(C)
    dEdC[:, :nact] = 4.0 * Y
    return {
        "E": E, "lam": lam, "Y": Y, "J": J, "K": K, "Hpp": Hpp, "D": D,
        "dEdn": pnof.grad_n(n, Hpp, J, K, npairs, ncwo, functional, nsingle), "dEdC": dEdC,
    }
