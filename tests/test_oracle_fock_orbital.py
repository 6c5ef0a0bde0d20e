"""Pins of the oracle's Fock vectors, Lagrangian, gradients and orbital step (CPU only)."""
import numpy as np
import pytest
import scipy.linalg

from oracle import pnof, stream
from tests import _brute
from tests._small import system

FUNCS = [pnof.PNOF5, pnof.PNOF7, pnof.PNOF7S]


def _setup(func, npairs=2, ncwo=2, nbf=9, naux=13, seed=3):
    s = system(nbf, naux, npairs, ncwo, seed=seed)
    n = pnof.on_sigmoid(s.gamma, npairs, ncwo)
    F = pnof.fock_ao(s.C, n, s.H, s.B, npairs, ncwo, func)
    return s, n, F


@pytest.mark.parametrize("func", FUNCS)
def test_euler_identity(func):
    """E = sum_p (n_p H_pp + lambda_pp): H is quadratic and V_ee quartic in the orbitals."""
    s, n, F = _setup(func)
    lam = pnof.lagrangian(s.C, F)
    nact = len(n)
    e = pnof.energy(s.C, n, s.H, s.B, 2, 2, func)
    hpp = pnof.h_no(s.C, s.H, nact)
    assert abs(e - np.sum(n * hpp + np.diag(lam)[:nact])) < 1e-12


@pytest.mark.parametrize("func", FUNCS)
def test_grad_C_central_differences(func):
    s, n, F = _setup(func)
    g = pnof.grad_C(s.C, F)
    h = 1e-5
    rng = np.random.default_rng(0)
    for _ in range(12):
        mu, q = rng.integers(0, 9), rng.integers(0, 6)
        Cp, Cm = s.C.copy(), s.C.copy()
        Cp[mu, q] += h
        Cm[mu, q] -= h
        fd = (pnof.energy(Cp, n, s.H, s.B, 2, 2, func) - pnof.energy(Cm, n, s.H, s.B, 2, 2, func)) / (2 * h)
        assert abs(fd - g[mu, q]) < 2e-8
    assert np.all(g[:, 6:] == 0)


@pytest.mark.parametrize("func", FUNCS)
def test_lagrangian_gradient_identity(func):
    """dE/dC = 4 F^q c_q = 4 C lambda for square orthogonal C."""
    s, n, F = _setup(func)
    lam = pnof.lagrangian(s.C, F)
    g = pnof.grad_C(s.C, F)
    assert np.max(np.abs(4 * s.C @ lam - g)) < 1e-13


@pytest.mark.parametrize("func", FUNCS)
def test_grad_n_central_differences(func):
    npairs, ncwo = 2, 2
    s, n, _ = _setup(func)
    nact = len(n)
    J, K = pnof.jk_no(s.B, s.C, nact, "df")
    hpp = pnof.h_no(s.C, s.H, nact)
    g = pnof.grad_n(n, hpp, J, K, npairs, ncwo, func)
    h = 1e-6
    for p in range(nact):
        e = np.zeros(nact)
        e[p] = h
        fd = (pnof.energy_from_jk(n + e, hpp, J, K, npairs, ncwo, func)
              - pnof.energy_from_jk(n - e, hpp, J, K, npairs, ncwo, func)) / (2 * h)
        assert abs(fd - g[p]) < 1e-8


@pytest.mark.parametrize("kind", ["sigmoid", "trig"])
def test_grad_gamma_chain_rule(kind):
    npairs, ncwo = 2, 2
    s = system(9, 13, npairs, ncwo)
    nact = 6
    J, K = pnof.jk_no(s.B, s.C, nact, "df")
    hpp = pnof.h_no(s.C, s.H, nact)
    rng = np.random.default_rng(5)
    if kind == "sigmoid":
        gam = rng.standard_normal(nact)
        nf, jf = pnof.on_sigmoid, pnof.on_sigmoid_jac
    else:
        gam = rng.uniform(0.2, 1.3, npairs * ncwo)
        nf, jf = pnof.on_trig, pnof.on_trig_jac
    n = nf(gam, npairs, ncwo)
    dg = jf(gam, npairs, ncwo).T @ pnof.grad_n(n, hpp, J, K, npairs, ncwo, pnof.PNOF7)
    h = 1e-6
    for r in range(len(gam)):
        e = np.zeros_like(gam)
        e[r] = h
        ep = pnof.energy_from_jk(nf(gam + e, npairs, ncwo), hpp, J, K, npairs, ncwo, pnof.PNOF7)
        em = pnof.energy_from_jk(nf(gam - e, npairs, ncwo), hpp, J, K, npairs, ncwo, pnof.PNOF7)
        assert abs((ep - em) / (2 * h) - dg[r]) < 1e-8


@pytest.mark.parametrize("func", FUNCS)
def test_stream_equals_definitional(func):
    npairs, ncwo = 2, 2
    s, n, F = _setup(func)
    lam = pnof.lagrangian(s.C, F)
    r = stream.lagrangian(s.C, n, s.H, s.B, npairs, ncwo, func, pchunk=4)
    e = pnof.energy(s.C, n, s.H, s.B, npairs, ncwo, func)
    assert abs(r["E"] - e) < 1e-12 * abs(e)
    assert np.max(np.abs(r["lam"] - lam)) < 1e-12
    assert np.max(np.abs(r["Y"] - pnof.fock_vectors(s.C, F))) < 1e-12
    assert np.max(np.abs(r["dEdC"] - pnof.grad_C(s.C, F))) < 1e-12


def test_hf_limit_lagrangian_is_hf_fock():
    """n in {0,1}: occupied columns of lambda are C^T F_HF C, virtual ones vanish."""
    npairs, ncwo = 3, 1
    s = system(8, 12, npairs, ncwo)
    n = np.zeros(6)
    n[:3] = 1.0
    F = pnof.fock_ao(s.C, n, s.H, s.B, npairs, ncwo, pnof.PNOF7)
    lam = pnof.lagrangian(s.C, F)
    ERI = pnof.eri_from_df(s.B)
    Fhf = _brute.rhf_fock(s.C, s.H, ERI, 3)
    ref = s.C.T @ Fhf @ s.C
    assert np.max(np.abs(lam[:, :3] - ref[:, :3])) < 1e-12
    assert np.max(np.abs(lam[:, 3:])) < 1e-15


def test_scf_solution_has_symmetric_lambda():
    """At a converged closed-shell SCF solution lambda is symmetric; its diagonal holds eps."""
    npairs, ncwo = 3, 1
    s = system(8, 12, npairs, ncwo, seed=4)
    ERI = pnof.eri_from_df(s.B)
    C, eps = _brute.rhf_scf(s.H, ERI, 3)
    n = np.zeros(6)
    n[:3] = 1.0
    F = pnof.fock_ao(C, n, s.H, ERI, npairs, ncwo, pnof.PNOF7, kind="eri")
    lam = pnof.lagrangian(C, F)
    occ = lam[:3, :3]
    assert np.max(np.abs(occ - occ.T)) < 1e-9
    assert np.max(np.abs(np.diag(lam)[:3] - eps[:3])) < 1e-9
    # lambda_pq - lambda_qp vanishes for occupied-virtual pairs too (Eq. lamlam)
    assert pnof.max_asym(lam) < 1e-8


# ------------------------------------------------------------------ orbital step
def test_orbital_step_eigendecomposition():
    s, n, F = _setup(pnof.PNOF7)
    lam = pnof.lagrangian(s.C, F)
    Cn, eps, S = pnof.orbital_step(lam, s.C)
    U = s.C.T @ Cn
    assert np.max(np.abs(S - S.T)) == 0.0
    assert np.max(np.abs(S @ U - U * eps[None, :])) < 1e-12
    assert np.max(np.abs(U.T @ U - np.eye(9))) < 1e-13
    assert np.max(np.abs(Cn.T @ Cn - np.eye(9))) < 1e-13      # orthonormality kept
    assert np.all(np.diff(eps) >= 0)
    assert np.max(np.abs(eps - scipy.linalg.eigh(S, eigvals_only=True, driver="ev"))) < 1e-12
    for j in range(9):
        i = np.argmax(np.abs(U[:, j]))
        assert U[i, j] > 0


def test_fockian_offdiagonals_and_zeta_scaling():
    rng = np.random.default_rng(8)
    lam = rng.standard_normal((6, 6))
    F = pnof.fockian_offdiag(lam)
    for q in range(6):
        for p in range(6):
            if q < p:
                assert F[q, p] == lam[p, q] - lam[q, p]       # Eq. Fockian, orientation of Eq. ene1
                assert F[p, q] == F[q, p]
            elif q == p:
                assert F[q, p] == 0.0
    zeta = 0.05
    Fs = pnof.scale_zeta(F, zeta)
    for p in range(6):
        for q in range(6):
            if p == q:
                continue
            x, k = F[p, q], 0
            while abs(x) > zeta:
                x /= 10.0
                k += 1
            assert Fs[p, q] == x and abs(Fs[p, q]) <= zeta
            assert k == 0 or abs(F[p, q]) / 10 ** (k - 1) > zeta
    diag = np.arange(6.0)
    Cn, eps, S = pnof.orbital_step(lam, np.eye(6), diag_prev=diag, zeta=zeta)
    assert np.all(np.diag(S) == diag)
    assert np.max(np.abs(S - S.T)) == 0.0


def test_scale_zeta_hand_worked_values():
    """zeta scaling of Section 3.2 (each off-diagonal element divided by ten while its magnitude
    exceeds zeta) on a fixed matrix, against values worked out by hand for zeta = 0.05:
    0.7 -> 0.07 -> 0.007 (two divisions), 12.5 -> 0.0125 (three), -0.0501 -> -0.00501 (one, sign
    kept), 0.05 stays (the test is strict: |F| > zeta), -0.004 and 0.0032 stay, the diagonal stays."""
    F = np.array([[9.0, 0.7, -0.004, 12.5],
                  [0.7, 8.0, 0.05, -0.0501],
                  [-0.004, 0.05, 7.0, 3.2e-3],
                  [12.5, -0.0501, 3.2e-3, 6.0]])
    want = np.array([[9.0, 0.007, -0.004, 0.0125],
                     [0.007, 8.0, 0.05, -0.00501],
                     [-0.004, 0.05, 7.0, 0.0032],
                     [0.0125, -0.00501, 0.0032, 6.0]])
    got = pnof.scale_zeta(F, 0.05)
    assert np.allclose(got, want, rtol=1e-14, atol=0.0)
    assert np.array_equal(np.diag(got), np.diag(F))
    assert got[1, 2] == 0.05   # the boundary value itself is not divided
