"""Pins of the oracle's integrals and energy (CPU only)."""
import math

import numpy as np
import pytest

import synth
from oracle import pnof, stream
from tests import _brute
from tests._small import system

FUNCS = [pnof.PNOF5, pnof.PNOF7, pnof.PNOF7S]


def test_eri_eightfold_symmetry():
    s = system(7, 11, 2, 1)
    E = pnof.eri_from_df(s.B)
    for perm in [(1, 0, 2, 3), (0, 1, 3, 2), (1, 0, 3, 2), (2, 3, 0, 1), (3, 2, 0, 1), (2, 3, 1, 0), (3, 2, 1, 0)]:
        assert np.max(np.abs(E - E.transpose(perm))) < 1e-15


@pytest.mark.parametrize("kind", ["eri", "df"])
def test_jk_match_brute_force_mo_integrals(kind):
    s = system(8, 12, 2, 2)
    nact = 6
    ERI = pnof.eri_from_df(s.B)
    mo = _brute.mo_eri(ERI, s.C[:, :nact])
    J, K = pnof.jk_no(ERI if kind == "eri" else s.B, s.C, nact, kind)
    Jb = np.array([[mo[p, p, q, q] for q in range(nact)] for p in range(nact)])
    Kb = np.array([[mo[p, q, p, q] for q in range(nact)] for p in range(nact)])
    assert np.max(np.abs(J - Jb)) < 1e-13
    assert np.max(np.abs(K - Kb)) < 1e-13
    assert np.max(np.abs(np.diag(K) - np.diag(J))) < 1e-13     # K_pp = J_pp
    assert np.max(np.abs(J - J.T)) < 1e-14 and np.max(np.abs(K - K.T)) < 1e-14
    assert np.all(K > -1e-15)                                   # sum_P b^2 >= 0


def test_jq_kq_symmetric_and_eri_equals_df():
    s = system(7, 10, 2, 1)
    ERI = pnof.eri_from_df(s.B)
    for q in range(4):
        J1, K1 = pnof.jk_ao_eri(ERI, s.C, q)
        J2, K2 = pnof.jk_ao_df(s.B, s.C, q)
        assert np.max(np.abs(J1 - J1.T)) < 1e-14 and np.max(np.abs(K1 - K1.T)) < 1e-14
        assert np.max(np.abs(J1 - J2)) < 1e-14 and np.max(np.abs(K1 - K2)) < 1e-14


def test_stream_jk_equals_definitional():
    s = system(9, 14, 2, 2)
    nact = 6
    J, K = pnof.jk_no(s.B, s.C, nact, "df")
    Js, Ks, _ = stream.jk(s.C, s.B, nact, pchunk=5)
    assert np.max(np.abs(J - Js)) < 1e-14 and np.max(np.abs(K - Ks)) < 1e-14


# ------------------------------------------------------------------ energies
@pytest.mark.parametrize("func", FUNCS)
def test_hf_limit_equals_textbook_rhf(func):
    """n_g = 1, weak n = 0: the closed-shell HF energy sum D (2H + 2J[D] - K[D])."""
    s = system(8, 12, 3, 1)
    npairs, ncwo = 3, 1
    n = np.zeros(6)
    n[:3] = 1.0
    ERI = pnof.eri_from_df(s.B)
    e = pnof.energy(s.C, n, s.H, ERI, npairs, ncwo, func, kind="eri")
    assert abs(e - _brute.rhf_energy(s.C, s.H, ERI, 3)) < 1e-12


@pytest.mark.parametrize("npairs,ncwo", [(1, 3), (2, 1), (2, 2), (3, 1)])
def test_pnof5_equals_apsg_expectation(npairs, ncwo):
    """PNOF5 is the energy of its generating APSG wavefunction (second quantisation)."""
    nact = npairs * (ncwo + 1)
    s = system(nact + 1, 13, npairs, ncwo, seed=11)
    n = pnof.on_sigmoid(s.gamma, npairs, ncwo)
    ERI = pnof.eri_from_df(s.B)
    pair, _ = pnof.layout(npairs, ncwo)
    members = [list(np.flatnonzero(pair[:nact] == g)) for g in range(npairs)]
    ref = _brute.apsg_energy(s.C, n, s.H, ERI, members, list(range(npairs)))
    e = pnof.energy(s.C, n, s.H, ERI, npairs, ncwo, pnof.PNOF5, kind="eri")
    assert abs(e - ref) < 1e-12


@pytest.mark.parametrize("func", FUNCS)
def test_energy_equals_reconstructed_2rdm_route(func):
    npairs, ncwo = 3, 1
    s = system(7, 12, npairs, ncwo, seed=5)
    n = pnof.on_sigmoid(s.gamma, npairs, ncwo)
    ERI = pnof.eri_from_df(s.B)
    pair, strong = pnof.layout(npairs, ncwo)
    ref = _brute.rdm2_energy(s.C, n, s.H, ERI, pair, strong, func)
    assert abs(pnof.energy(s.C, n, s.H, ERI, npairs, ncwo, func, kind="eri") - ref) < 1e-12


def test_one_pair_functionals_coincide():
    s = system(6, 10, 1, 3)
    n = pnof.on_sigmoid(s.gamma, 1, 3)
    es = [pnof.energy(s.C, n, s.H, s.B, 1, 3, f) for f in FUNCS]
    assert max(es) - min(es) < 1e-13


def test_pnof7s_equals_pnof7_at_half_filling():
    npairs, ncwo = 3, 1
    s = system(8, 12, npairs, ncwo)
    n = np.full(6, 0.5)
    e7 = pnof.energy(s.C, n, s.H, s.B, npairs, ncwo, pnof.PNOF7)
    e7s = pnof.energy(s.C, n, s.H, s.B, npairs, ncwo, pnof.PNOF7S)
    e5 = pnof.energy(s.C, n, s.H, s.B, npairs, ncwo, pnof.PNOF5)
    assert abs(e7 - e7s) < 1e-13
    assert abs(e7 - e5) > 1e-6          # the Phi term is present


def _embed_fragments(fa, fb, npairs_a, npairs_b, ncwo):
    """Direct sum of two fragments with disjoint AO blocks and disjoint P support."""
    na, nb = fa.wl.nbf, fb.wl.nbf
    Pa, Pb = fa.B.shape[0], fb.B.shape[0]
    n = na + nb
    B = np.zeros((Pa + Pb, n, n))
    B[:Pa, :na, :na] = fa.B
    B[Pa:, na:, na:] = fb.B
    H = np.zeros((n, n))
    H[:na, :na] = fa.H
    H[na:, na:] = fb.H
    npairs = npairs_a + npairs_b
    la, _ = pnof.layout(npairs_a, ncwo, na)
    lb, _ = pnof.layout(npairs_b, ncwo, nb)
    l, _ = pnof.layout(npairs, ncwo, n)
    na_act, nb_act = npairs_a * (ncwo + 1), npairs_b * (ncwo + 1)
    C = np.zeros((n, n))
    nvec = np.zeros(npairs * (ncwo + 1))
    gam_a = pnof.on_sigmoid(fa.gamma, npairs_a, ncwo)
    gam_b = pnof.on_sigmoid(fb.gamma, npairs_b, ncwo)
    used_a, used_b = set(), set()
    for g in range(npairs):
        tgt = list(np.flatnonzero(l == g))
        if g < npairs_a:
            src = list(np.flatnonzero(la == g))
            for t, sidx in zip(tgt, src):
                C[:na, t] = fa.C[:, sidx]
                nvec[t] = gam_a[sidx]
                used_a.add(sidx)
        else:
            src = list(np.flatnonzero(lb == g - npairs_a))
            for t, sidx in zip(tgt, src):
                C[na:, t] = fb.C[:, sidx]
                nvec[t] = gam_b[sidx]
                used_b.add(sidx)
    # remaining columns: the fragments' inactive orbitals
    rest = [c for c in range(n) if not np.any(C[:, c])]
    extra = [("a", c) for c in range(na) if c not in used_a] + [("b", c) for c in range(nb) if c not in used_b]
    for t, (f, c) in zip(rest, extra):
        if f == "a":
            C[:na, t] = fa.C[:, c]
        else:
            C[na:, t] = fb.C[:, c]
    return C, nvec, H, B, gam_a, gam_b


@pytest.mark.parametrize("func", FUNCS)
def test_additivity_of_separated_fragments(func):
    """Size consistency: non-interacting fragments add (synthetic analogue of the 1000 A water)."""
    ncwo = 1
    fa = system(6, 9, 2, ncwo, seed=21)
    fb = system(5, 8, 1, ncwo, seed=22)
    C, n, H, B, na_, nb_ = _embed_fragments(fa, fb, 2, 1, ncwo)
    assert np.max(np.abs(C.T @ C - np.eye(C.shape[0]))) < 1e-14
    e = pnof.energy(C, n, H, B, 3, ncwo, func)
    ea = pnof.energy(fa.C, na_, fa.H, fa.B, 2, ncwo, func)
    eb = pnof.energy(fb.C, nb_, fb.H, fb.B, 1, ncwo, func)
    assert abs(e - (ea + eb)) < 1e-12


@pytest.mark.parametrize("func", FUNCS)
def test_invariances(func):
    npairs, ncwo = 2, 2
    s = system(8, 12, npairs, ncwo)
    n = pnof.on_sigmoid(s.gamma, npairs, ncwo)
    e0 = pnof.energy(s.C, n, s.H, s.B, npairs, ncwo, func)
    # sign of one orbital
    C2 = s.C.copy()
    C2[:, 3] *= -1
    assert abs(pnof.energy(C2, n, s.H, s.B, npairs, ncwo, func) - e0) < 1e-12
    # AO rotation applied to (B_P, H, C)
    R, _ = np.linalg.qr(np.random.default_rng(9).standard_normal((8, 8)))
    Br = np.einsum("mi,Pmn,nj->Pij", R, s.B, R)
    e1 = pnof.energy(R.T @ s.C, n, R.T @ s.H @ R, Br, npairs, ncwo, func)
    assert abs(e1 - e0) < 1e-12
    # relabelling the two weak orbitals of a pair together with their ONs
    pair, strong = pnof.layout(npairs, ncwo)
    w = [p for p in range(6) if pair[p] == 0 and not strong[p]]
    C3, n3 = s.C.copy(), n.copy()
    C3[:, [w[0], w[1]]] = C3[:, [w[1], w[0]]]
    n3[[w[0], w[1]]] = n3[[w[1], w[0]]]
    assert abs(pnof.energy(C3, n3, s.H, s.B, npairs, ncwo, func) - e0) < 1e-12


def test_sigmoid_energy_is_not_trivial():
    """Guard: the two-electron part of the small test systems is not negligible."""
    npairs, ncwo = 2, 2
    s = system(8, 12, npairs, ncwo)
    n = pnof.on_sigmoid(s.gamma, npairs, ncwo)
    J, K = pnof.jk_no(s.B, s.C, 6, "df")
    e2 = pnof.energy_from_jk(n, np.zeros(6), J, K, npairs, ncwo, pnof.PNOF7)
    assert abs(e2) > 1e-2
