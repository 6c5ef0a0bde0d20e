"""Pins of the oracle's optimisation loops (Sections 3.1-3.4), CPU only.

* Occupation optimisation: for one pair with one weak orbital every functional is the two-electron
  energy of the Loewdin-Shull form sqrt(n_g)|g gbar> - sqrt(n_w)|w wbar>, whose minimum over the
  occupations is the lowest eigenvalue of the 2 x 2 pair-CI matrix in the fixed orbitals.
* Orbital step: one diagonalisation of the matrix of Eq. Fockian with an increasing diagonal lowers
  the energy (first-order statement of Eq. ene1).
* Orbital loop, Hartree-Fock limit: with occupations fixed at 1 (strong) and 0 (weak) the loop of
  Section 3.4 reaches the textbook closed-shell SCF energy (level-shifted Roothaan iterations).
* Full loop: the energy decreases from the guess and lambda becomes symmetric (Section 3.4).
"""
import numpy as np
import pytest
from scipy.linalg import expm

from oracle import optimize, pnof, stream
from tests import _brute
from tests._small import eri, system

FUNCS = [pnof.PNOF5, pnof.PNOF7, pnof.PNOF7S]


@pytest.mark.parametrize("func", FUNCS)
@pytest.mark.parametrize("kind", ["sigmoid", "trig"])
def test_one_pair_occupations_give_pair_ci(func, kind):
    s = system(6, 24, 1, 1, seed=11)
    Hpp = pnof.h_no(s.C, s.H, 2)
    J, K = pnof.jk_no(s.B, s.C, 2, "df")
    g, w = 0, pnof.weak_orbitals(0, 1, 1)[0]
    M = np.array([[2 * Hpp[g] + J[g, g], K[g, w]], [K[g, w], 2 * Hpp[w] + J[w, w]]])
    e_ci = np.linalg.eigvalsh(M)[0]
    gamma0 = np.zeros(2) if kind == "sigmoid" else np.array([0.3])
    gamma, E, _ = optimize.optimize_on(gamma0, Hpp, J, K, 1, 1, func, kind)
    # the sign convention (strong +, weak -) reaches the ground state because K_gw > 0
    assert K[g, w] > 0
    assert abs(E - e_ci) < 1e-10


@pytest.mark.parametrize("kind", ["sigmoid", "trig"])
def test_occupation_optimum_is_stationary(kind):
    s = system(12, 48, 2, 3, seed=12)
    nact = 8
    Hpp = pnof.h_no(s.C, s.H, nact)
    J, K = pnof.jk_no(s.B, s.C, nact, "df")
    gamma0 = s.gamma if kind == "sigmoid" else np.full(2 * 3, 0.4)
    gamma, E, _ = optimize.optimize_on(gamma0, Hpp, J, K, 2, 3, pnof.PNOF7, kind)
    E0, _ = optimize.on_energy_grad(gamma0, Hpp, J, K, 2, 3, pnof.PNOF7, kind)
    assert E <= E0
    # central differences of the energy vanish at the optimum
    h = 1e-5
    for r in range(len(gamma)):
        gp, gm = gamma.copy(), gamma.copy()
        gp[r] += h
        gm[r] -= h
        fd = (optimize.on_energy_grad(gp, Hpp, J, K, 2, 3, pnof.PNOF7, kind)[0]
              - optimize.on_energy_grad(gm, Hpp, J, K, 2, 3, pnof.PNOF7, kind)[0]) / (2 * h)
        assert abs(fd) < 1e-6
    n = optimize.on_map(gamma, 2, 3, kind)
    pair, _ = pnof.layout(2, 3)
    for gidx in range(2):
        assert abs(np.sum(n[pair == gidx]) - 1.0) < 1e-14


@pytest.mark.filterwarnings("ignore::RuntimeWarning")
def test_fockian_step_descends():
    """From orbitals near the closed-shell solution, one step with the orbital energies as the
    (increasing) diagonal lowers the energy, as Eq. ene1 states for the aufbau choice."""
    s = system(10, 40, 2, 2, seed=3)
    ERI = eri(s)
    Cs, eps = _brute.rhf_scf(s.H, ERI, 2)
    n = np.zeros(6)
    n[:2] = 1.0
    rng = np.random.default_rng(0)
    A = rng.standard_normal((10, 10))
    C = Cs @ expm(0.02 * (A - A.T))
    r0 = stream.lagrangian(C, n, s.H, s.B, 2, 2, pnof.PNOF7)
    C1, _, _ = pnof.orbital_step(r0["lam"], C, diag_prev=eps)
    r1 = stream.lagrangian(C1, n, s.H, s.B, 2, 2, pnof.PNOF7)
    assert r1["E"] < r0["E"] - 1e-3


@pytest.mark.filterwarnings("ignore::RuntimeWarning")
def test_hartree_fock_limit_of_the_orbital_loop():
    s = system(10, 40, 2, 2, seed=3)
    ERI = eri(s)
    Cs, _ = _brute.rhf_scf(s.H, ERI, 2)
    e_rhf = _brute.rhf_energy(Cs, s.H, ERI, 2)
    n = np.zeros(6)
    n[:2] = 1.0
    C0 = np.linalg.eigh(s.H)[1]
    r = optimize.optimize(C0, None, s.H, s.B, 2, 2, fixed_n=n, delta=1e-7, eps_n=0, eps_phi=0, eps=0,
                          maxit=400)
    assert r["converged"] and r["max_asym"] < 1e-7
    assert abs(r["E"] - e_rhf) < 1e-9


@pytest.mark.parametrize("ndiis,zeta", [(0, 0.0), (0, 0.1), (4, 0.0)])
def test_full_loop_descends_and_symmetrises(ndiis, zeta):
    s = system(10, 40, 2, 2, seed=3)
    C0 = np.linalg.eigh(s.H)[1]
    r = optimize.optimize(C0, s.gamma, s.H, s.B, 2, 2, delta=1e-5, eps_n=0, eps_phi=0, eps=0, maxit=600,
                          ndiis=ndiis, zeta=zeta)
    assert r["converged"] and r["max_asym"] < 1e-5
    assert r["E"] < r["history"][0]
    # the final occupations satisfy the pairing sum rule
    pair, _ = pnof.layout(2, 2)
    for g in range(2):
        assert abs(np.sum(r["n"][pair == g]) - 1.0) < 1e-14


def test_diis_reaches_the_same_solution_faster():
    """DIIS (Section 3.3), with the matrices combined in the fixed AO basis, converges to the same
    stationary point as the plain iteration, in fewer steps."""
    s = system(10, 40, 2, 2, seed=3)
    C0 = np.linalg.eigh(s.H)[1]
    kw = dict(delta=1e-6, eps_n=0, eps_phi=0, eps=0, maxit=800)
    plain = optimize.optimize(C0, s.gamma, s.H, s.B, 2, 2, ndiis=0, **kw)
    diis = optimize.optimize(C0, s.gamma, s.H, s.B, 2, 2, ndiis=4, **kw)
    assert plain["converged"] and diis["converged"]
    assert diis["iterations"] < plain["iterations"]
    assert abs(diis["E"] - plain["E"]) < 1e-8


def test_diis_coefficients_solve_the_constrained_least_squares():
    """sum c_j = 1 and the combination minimises |sum c_j e^j| (checked against a direct
    minimisation over the affine set)."""
    rng = np.random.default_rng(4)
    errs = [rng.standard_normal((5, 5)) for _ in range(3)]
    mats = [np.eye(5) * (j + 1) for j in range(3)]
    F = optimize.diis_extrapolate(mats, errs)
    c = np.diag(F)[0] - 1.0          # F = sum c_j (j+1) I with sum c_j = 1 -> c_1 + 2 c_2 = F_00 - 1
    E = np.array([e.ravel() for e in errs]).T
    # parametrise c = (1 - a - b, a, b) and minimise |E c| by least squares
    A = np.stack([E[:, 1] - E[:, 0], E[:, 2] - E[:, 0]], axis=1)
    ab, *_ = np.linalg.lstsq(A, -E[:, 0], rcond=None)
    assert abs(c - (ab[0] + 2 * ab[1])) < 1e-12
