"""Pins of the NOF-MP2 reference terms (Section 4, Eqs. HFL and Esta), CPU only.

* E_hf is the closed-shell Hartree-Fock energy of the strong natural orbitals, whatever the
  occupations (textbook formula sum D (2H + 2J[D] - K[D]) with D = sum_g c_g c_g^T).
* In the Hartree-Fock limit (n = 1 strong, 0 weak) E_sta vanishes and E_hf equals the PNOF energy.
* The inter-subspace part of E_sta is the difference between the PNOF7s and PNOF5 energies
  (Eq. Efg_s against Eq. Efg with Phi = 0), for any occupations.
* With every occupation 1/2 (Lambda = 1) the intra-subspace part is the off-diagonal intrapair
  sum of Eq. Eg.
"""
import numpy as np

from oracle import pnof
from tests import _brute
from tests._small import eri, sigmoid_n, system


def _jk(s, nact):
    J, K = pnof.jk_no(s.B, s.C, nact, "df")
    return pnof.h_no(s.C, s.H, nact), J, K


def test_e_hf_is_textbook_rhf_of_strong_orbitals():
    s = system(9, 30, 2, 2, seed=21)
    n = sigmoid_n(s)
    Hpp, J, K = _jk(s, 6)
    E_hf, _ = pnof.nofmp2_reference(n, Hpp, J, K, 2, 2)
    assert abs(E_hf - _brute.rhf_energy(s.C, s.H, eri(s), 2)) < 1e-11


def test_hartree_fock_limit():
    s = system(9, 30, 2, 2, seed=22)
    n = np.zeros(6)
    n[:2] = 1.0
    Hpp, J, K = _jk(s, 6)
    E_hf, E_sta = pnof.nofmp2_reference(n, Hpp, J, K, 2, 2)
    assert E_sta == 0.0
    for func in (pnof.PNOF5, pnof.PNOF7, pnof.PNOF7S):
        assert abs(E_hf - pnof.energy_from_jk(n, Hpp, J, K, 2, 2, func)) < 1e-11


def test_inter_subspace_static_term_is_pnof7s_minus_pnof5():
    s = system(10, 40, 3, 2, seed=23)
    rng = np.random.default_rng(5)
    n = pnof.on_sigmoid(rng.standard_normal(9), 3, 2)
    Hpp, J, K = _jk(s, 9)
    _, E_sta = pnof.nofmp2_reference(n, Hpp, J, K, 3, 2)
    # remove the intra-subspace part by zeroing K inside the subspaces
    pair, _ = pnof.layout(3, 2)
    Kx = K.copy()
    for p in range(9):
        for q in range(9):
            if p != q and pair[p] == pair[q]:
                Kx[p, q] = 0.0
    _, E_inter = pnof.nofmp2_reference(n, Hpp, J, Kx, 3, 2)
    d = pnof.energy_from_jk(n, Hpp, J, K, 3, 2, pnof.PNOF7S) - pnof.energy_from_jk(n, Hpp, J, K, 3, 2, pnof.PNOF5)
    assert abs(E_inter - d) < 1e-12


def test_half_filling_intra_term():
    s = system(8, 30, 2, 1, seed=24)
    n = np.full(4, 0.5)
    Hpp, J, K = _jk(s, 4)
    _, E_sta = pnof.nofmp2_reference(n, Hpp, J, K, 2, 1)
    # Lambda = 1 and Phi^2 = 1/4: intrapair off-diagonal of Eq. Eg, minus 1/4 of the inter K sum
    pair, strong = pnof.layout(2, 1)
    intra = sum(-0.5 * K[p, q] for p in range(4) for q in range(4) if p != q and pair[p] == pair[q])
    inter = sum(-0.25 * K[p, q] for p in range(4) for q in range(4) if pair[p] != pair[q])
    assert abs(E_sta - (intra + inter)) < 1e-12
