"""Oracle of the two optimisation loops of Section 3 (test infrastructure only).

* ``optimize_on``: occupation optimisation at fixed orbitals (Section 3.1).  E is minimised over
  the unconstrained auxiliary variables gamma (Eqs. soo, woo, or the sigmoid map) with a
  quasi-Newton method; only H_pp, J and K of the fixed orbitals enter, as stated at the end of
  Section 3.4 (the integral transformation is done once per occupation optimisation).
* ``optimize``: the computational procedure of Section 3.4.
  - Initial step: occupation optimisation with the guess orbitals, then one diagonalisation of
    the symmetrised Lagrangian, whose eigenvalues become the first diagonal of the matrix of
    Eq. Fockian.
  - Iterations j: occupations for fixed orbitals; the matrix of Eq. Fockian with the previous
    diagonal; off-diagonal scaling by zeta (Section 3.2); DIIS extrapolation with the
    off-diagonal elements as error vectors (Section 3.3); diagonalisation; new diagonal.
  - Convergence: the three energy differences epsilon_n, epsilon_phi, epsilon and the symmetry
    of lambda, delta (Section 3.4).

The quasi-Newton minimiser is scipy's L-BFGS-B, used as a library primitive.  The eigensolver is
numpy's LAPACK ``eigh``.
"""
from __future__ import annotations

import math

import numpy as np

from . import pnof, stream


def on_map(gamma, npairs, ncwo, kind="sigmoid", nsingle=0):
    if kind == "sigmoid":
        return pnof.on_sigmoid(gamma, npairs, ncwo, nsingle)
    return pnof.on_trig(gamma, npairs, ncwo, nsingle)


def on_jac(gamma, npairs, ncwo, kind="sigmoid", nsingle=0):
    if kind == "sigmoid":
        return pnof.on_sigmoid_jac(gamma, npairs, ncwo, nsingle)
    return pnof.on_trig_jac(gamma, npairs, ncwo, nsingle)


def on_energy_grad(gamma, Hpp, J, K, npairs, ncwo, functional=pnof.PNOF7, kind="sigmoid", nsingle=0):
    """E(n(gamma)) at fixed J, K, H_pp and its gradient (dn/dgamma)^T dE/dn."""
    n = on_map(gamma, npairs, ncwo, kind, nsingle)
    E = pnof.energy_from_jk(n, Hpp, J, K, npairs, ncwo, functional, nsingle)
    g = on_jac(gamma, npairs, ncwo, kind, nsingle).T @ pnof.grad_n(n, Hpp, J, K, npairs, ncwo, functional, nsingle)
    return E, g


def optimize_on(gamma0, Hpp, J, K, npairs, ncwo, functional=pnof.PNOF7, kind="sigmoid", gtol=1e-10,
                maxiter=1000, nsingle=0):
    """Minimise E over gamma at fixed orbitals; returns (gamma, E, iterations)."""
    from scipy.optimize import minimize

    res = minimize(on_energy_grad, np.asarray(gamma0, dtype=np.float64), jac=True, method="L-BFGS-B",
                   args=(Hpp, J, K, npairs, ncwo, functional, kind, nsingle),
                   options={"gtol": gtol, "ftol": 1e-15, "maxiter": maxiter, "maxcor": 10})
    return res.x, float(res.fun), int(res.nit)


def _jk_hpp(C, H, ints, nact, kind):
    J, K = pnof.jk_no(ints, C, nact, kind)
    return pnof.h_no(C, H, nact), J, K


def _lagrangian(C, n, H, ints, npairs, ncwo, functional, kind, nsingle=0):
    if kind == "df":
        r = stream.lagrangian(C, n, H, ints, npairs, ncwo, functional, nsingle=nsingle)
        return r["E"], r["lam"]
    F = pnof.fock_ao(C, n, H, ints, npairs, ncwo, functional, kind, nsingle)
    lam = pnof.lagrangian(C, F)
    return pnof.energy(C, n, H, ints, npairs, ncwo, functional, kind, nsingle), lam


def diis_extrapolate(mats, errs):
    """F = sum_j c_j F^j with sum_j c_j = 1 minimising |sum_j c_j e^j| (Section 3.3, Pulay)."""
    m = len(mats)
    Bm = np.zeros((m + 1, m + 1))
    for i in range(m):
        for j in range(m):
            Bm[i, j] = float(np.sum(errs[i] * errs[j]))
    Bm[:m, m] = -1.0
    Bm[m, :m] = -1.0
    rhs = np.zeros(m + 1)
    rhs[m] = -1.0
    c = np.linalg.solve(Bm, rhs)[:m]
    return sum(ci * Fi for ci, Fi in zip(c, mats))


def optimize(C0, gamma0, H, ints, npairs, ncwo, functional=pnof.PNOF7, kind="df", on_kind="sigmoid",
             maxit=200, eps_n=1e-10, eps_phi=1e-10, eps=1e-10, delta=1e-4, zeta=0.0, ndiis=0, fixed_n=None,
             nsingle=0):
    """Orbital + occupation optimisation of Section 3.4.

    fixed_n: occupations held fixed (no occupation optimisation), e.g. the Hartree-Fock limit.
    Returns dict(C, gamma, n, E, max_asym, iterations, converged, history).
    """
    nact = npairs * (ncwo + 1) + nsingle
    C = np.array(C0, dtype=np.float64)
    gamma = None if gamma0 is None else np.array(gamma0, dtype=np.float64)

    def occupations(C, gamma):
        if fixed_n is not None:
            n = np.asarray(fixed_n, dtype=np.float64)
            Hpp, J, K = _jk_hpp(C, H, ints, nact, kind)
            return gamma, n, pnof.energy_from_jk(n, Hpp, J, K, npairs, ncwo, functional, nsingle)
        Hpp, J, K = _jk_hpp(C, H, ints, nact, kind)
        gamma, E, _ = optimize_on(gamma, Hpp, J, K, npairs, ncwo, functional, on_kind, nsingle=nsingle)
        return gamma, on_map(gamma, npairs, ncwo, on_kind, nsingle), E

    # initial step
    gamma, n, _ = occupations(C, gamma)
    E0, lam = _lagrangian(C, n, H, ints, npairs, ncwo, functional, kind, nsingle)
    C, diag, _ = pnof.orbital_step(lam, C)
    E_prev, lam = _lagrangian(C, n, H, ints, npairs, ncwo, functional, kind, nsingle)
    history = [E0, E_prev]
    crit = {}
    mats, errs = [], []
    converged = False
    it = 0
    for it in range(1, maxit + 1):
        gamma, n, E_n = occupations(C, gamma)          # E[n^{j+1}, phi^j]
        E_fixed_orb, lam = _lagrangian(C, n, H, ints, npairs, ncwo, functional, kind, nsingle)
        # matrix of Eq. Fockian: off-diagonal from lambda, diagonal from the previous step
        F = pnof.fockian_offdiag(lam)
        if zeta > 0:
            F = pnof.scale_zeta(F, zeta)
        F[np.diag_indices(F.shape[0])] = diag
        if ndiis > 1:
            # the matrices of successive steps live in different orbital bases: they are stored
            # and combined in the fixed AO basis (F_AO = C F C^T, S = I), then brought back
            mats.append(C @ F @ C.T)
            errs.append(C @ (F - np.diag(np.diag(F))) @ C.T)
            mats, errs = mats[-ndiis:], errs[-ndiis:]
            if len(mats) >= 2:
                F = C.T @ diis_extrapolate(mats, errs) @ C
        diag, U = np.linalg.eigh(F)
        C = C @ pnof.sign_fix(U)
        E_new, lam_new = _lagrangian(C, n, H, ints, npairs, ncwo, functional, kind, nsingle)
        history.append(E_new)
        crit = {"d_n": abs(E_n - E_prev), "d_phi": abs(E_new - E_fixed_orb), "d_E": abs(E_new - E_prev),
                "max_asym": pnof.max_asym(lam_new)}
        E_prev = E_new
        # the symmetry of lambda prevails over the three energy criteria (Section 3.4)
        if crit["max_asym"] < delta:
            converged = True
            break
        if crit["d_n"] < eps_n and crit["d_phi"] < eps_phi and crit["d_E"] < eps:
            break
    _, lam = _lagrangian(C, n, H, ints, npairs, ncwo, functional, kind, nsingle)
    return {"C": C, "gamma": gamma, "n": n, "E": E_prev, "max_asym": pnof.max_asym(lam), "iterations": it,
            "converged": converged, "history": history, "criteria": crit}
