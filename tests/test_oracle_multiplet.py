"""Pins of the multiplet extension (Section 2: N_I singly occupied orbitals, S = N_I/2), CPU only.

* Restricted open-shell limit: strong n = 1, weak n = 0, single n = 1/2.  PNOF7 and PNOF7s give the
  energy of the high-spin determinant (closed shells doubly occupied, singles with alpha spin),
  computed by second quantisation; PNOF5 (Phi = 0) does so only with one single orbital.
* The energy equals the explicit spin-blocked 2RDM route with the Omega_I rules (no intra term for a
  single orbital; exchange form of the Phi term between two single orbitals), for correlated
  occupations and every functional.
* Euler identity and dE/dC by central differences with single orbitals present.
* Sum rule 2 sum n = N_II + N_I; the NOF-MP2 HF-like energy with singles is the closed-shell-like
  energy sum D (H + J[D]/2 - K[D]/4) of the AO density D = sum_g 2 A_g c_g c_g^T (A = 1 strong,
  1/2 single) minus the self-Coulomb J_gg/4 of each single orbital (Eq. HFL and the closed-shell-like
  Fock operator of Section 4).  This differs from the high-spin determinant energy by half the
  exchange between single orbitals.
"""
import numpy as np
import pytest

from oracle import pnof
from tests import _brute
from tests._small import eri, system

FUNCS = [pnof.PNOF5, pnof.PNOF7, pnof.PNOF7S]
NP, NG, NS = 2, 1, 2          # 2 pairs with one weak orbital each, 2 single electrons (triplet)
NACT = NP * (NG + 1) + NS


def _occupations(s, seed=0):
    gamma = np.random.default_rng(seed).standard_normal(NACT)
    return pnof.on_sigmoid(gamma, NP, NG, NS)


@pytest.mark.parametrize("func", FUNCS)
@pytest.mark.parametrize("nsingle", [1, 2])
def test_restricted_open_shell_limit(func, nsingle):
    s = system(8, 30, NP, NG, seed=31)
    nact = NP * (NG + 1) + nsingle
    n = np.zeros(nact)
    n[:NP] = 1.0
    n[NP:NP + nsingle] = 0.5
    E = pnof.energy(s.C, n, s.H, s.B, NP, NG, func, nsingle=nsingle)
    closed = list(range(NP))
    singles = list(range(NP, NP + nsingle))
    E_det = _brute.determinant_energy(s.C, s.H, eri(s), closed + singles, closed)
    if func == pnof.PNOF5 and nsingle > 1:
        assert abs(E - E_det) > 1e-6          # Phi = 0 misses half of the single-single exchange
    else:
        assert abs(E - E_det) < 1e-11


@pytest.mark.parametrize("func", FUNCS)
def test_energy_equals_2rdm_route_with_singles(func):
    s = system(9, 30, NP, NG, seed=32)
    n = _occupations(s)
    pair, strong = pnof.layout(NP, NG, nsingle=NS)
    E = pnof.energy(s.C, n, s.H, s.B, NP, NG, func, nsingle=NS)
    E2 = _brute.rdm2_energy(s.C, n, s.H, eri(s), pair, strong, func, singles=pnof.single_orbitals(NP, NS))
    assert abs(E - E2) < 1e-11


@pytest.mark.parametrize("func", FUNCS)
def test_euler_identity_and_gradient_with_singles(func):
    s = system(9, 30, NP, NG, seed=33)
    n = _occupations(s)
    F = pnof.fock_ao(s.C, n, s.H, s.B, NP, NG, func, nsingle=NS)
    lam = pnof.lagrangian(s.C, F)
    E = pnof.energy(s.C, n, s.H, s.B, NP, NG, func, nsingle=NS)
    assert abs(E - np.sum(n * pnof.h_no(s.C, s.H, NACT) + np.diag(lam)[:NACT])) < 1e-12
    g = pnof.grad_C(s.C, F)
    h = 1e-5
    for mu, q in [(0, 2), (3, 3), (5, 1), (8, 5)]:
        Cp, Cm = s.C.copy(), s.C.copy()
        Cp[mu, q] += h
        Cm[mu, q] -= h
        fd = (pnof.energy(Cp, n, s.H, s.B, NP, NG, func, nsingle=NS)
              - pnof.energy(Cm, n, s.H, s.B, NP, NG, func, nsingle=NS)) / (2 * h)
        assert abs(fd - g[mu, q]) < 1e-7


def test_layout_and_sum_rule_with_singles():
    pair, strong = pnof.layout(3, 2, nsingle=2)
    assert list(pair[:5]) == [0, 1, 2, 3, 4]          # strong orbitals, then the singles
    assert [pnof.weak_orbitals(g, 3, 2, 2) for g in range(3)] == [[9, 10], [7, 8], [5, 6]]
    rng = np.random.default_rng(1)
    for n in (pnof.on_sigmoid(rng.standard_normal(11), 3, 2, 2), pnof.on_trig(rng.standard_normal(6), 3, 2, 2)):
        assert abs(2 * np.sum(n) - (2 * 3 + 2)) < 1e-13
        assert n[3] == 0.5 and n[4] == 0.5


def test_grad_n_with_singles_central_differences():
    s = system(9, 30, NP, NG, seed=34)
    n = _occupations(s)
    Hpp = pnof.h_no(s.C, s.H, NACT)
    J, K = pnof.jk_no(s.B, s.C, NACT, "df")
    g = pnof.grad_n(n, Hpp, J, K, NP, NG, pnof.PNOF7, NS)
    h = 1e-6
    for p in range(NACT):
        npl, nmi = n.copy(), n.copy()
        npl[p] += h
        nmi[p] -= h
        fd = (pnof.energy_from_jk(npl, Hpp, J, K, NP, NG, pnof.PNOF7, NS)
              - pnof.energy_from_jk(nmi, Hpp, J, K, NP, NG, pnof.PNOF7, NS)) / (2 * h)
        assert abs(fd - g[p]) < 1e-6


def test_nofmp2_hf_like_energy_with_singles():
    s = system(8, 30, NP, NG, seed=35)
    n = _occupations(s)
    Hpp = pnof.h_no(s.C, s.H, NACT)
    J, K = pnof.jk_no(s.B, s.C, NACT, "df")
    E_hf, _ = pnof.nofmp2_reference(n, Hpp, J, K, NP, NG, NS)
    ERI = eri(s)
    A = [1.0] * NP + [0.5] * NS
    D = sum(2 * a * np.outer(s.C[:, g], s.C[:, g]) for g, a in enumerate(A))
    JD = np.einsum("mnls,ls->mn", ERI, D)
    KD = np.einsum("mlns,ls->mn", ERI, D)
    E_ref = float(np.sum(D * (s.H + 0.5 * JD - 0.25 * KD)))
    for t in range(NP, NP + NS):
        E_ref -= 0.25 * J[t, t]
    assert abs(E_hf - E_ref) < 1e-11
    closed = list(range(NP))
    E_det = _brute.determinant_energy(s.C, s.H, ERI, closed + list(range(NP, NP + NS)), closed)
    assert abs((E_hf - E_det) - 0.5 * K[NP, NP + 1]) < 1e-11
