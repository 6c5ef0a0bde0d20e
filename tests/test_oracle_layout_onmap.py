"""Pins of the oracle's orbital layout and occupation-number maps (CPU only)."""
import math
import os

import numpy as np
import pytest

from oracle import pnof

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _table(name):
    rows = [l.split() for l in open(os.path.join(GOLDEN, name)) if l.strip() and not l.startswith("#")]
    return np.array([[float(x) for x in r[1:]] for r in rows])


def _pair_sums(occ2, npairs, ncwo, offset=0):
    pair, _ = pnof.layout(npairs, ncwo)
    sums = np.zeros((npairs, occ2.shape[1]))
    for p in range(npairs * (ncwo + 1)):
        sums[pair[p]] += occ2[offset + p]
    return sums


def test_layout_table1_pairs_sum_to_two():
    """Water, N_g = 4 (Table 1): every subspace holds two electrons under the layout."""
    t = _table("water_ons_table1.txt")
    sums = _pair_sums(t, npairs=5, ncwo=4)
    # 5 entries per subspace, each rounded to 1e-3
    assert np.max(np.abs(sums - 2.0)) <= 5 * 0.0005 + 1e-12


def test_layout_table1_rejects_interleaved_coupling():
    """The same table violates the sum rule under an interleaved weak-orbital coupling."""
    t = _table("water_ons_table1.txt")
    npairs, ncwo = 5, 4
    sums = np.zeros((npairs, t.shape[1]))
    for g in range(npairs):
        sums[g] += t[g]
        for k in range(ncwo):
            sums[g] += t[npairs + k * npairs + (npairs - 1 - g)]
    assert np.max(np.abs(sums - 2.0)) > 0.005


def test_layout_table2_pairs_sum_to_two():
    """Water, N_g = 1 (Table 2), orbital 1 frozen: pairs (5,6), (4,7), (3,8), (2,9)."""
    t = _table("water_ons_table2.txt")
    sums = _pair_sums(t, npairs=4, ncwo=1, offset=1)
    assert np.max(np.abs(sums - 2.0)) <= 2 * 0.000005 + 1e-12


@pytest.mark.parametrize("npairs,ncwo", [(1, 1), (3, 2), (5, 4), (4, 1)])
def test_layout_partition(npairs, ncwo):
    pair, strong = pnof.layout(npairs, ncwo, nbf=npairs * (ncwo + 1) + 3)
    nact = npairs * (ncwo + 1)
    assert list(pair[nact:]) == [-1, -1, -1]
    for g in range(npairs):
        members = np.flatnonzero(pair == g)
        assert len(members) == ncwo + 1
        assert strong[g] and pair[g] == g
        assert sum(strong[members]) == 1


# ------------------------------------------------------------------ sigmoid map
def test_sigmoid_sum_rule_and_bounds():
    rng = np.random.default_rng(1)
    npairs, ncwo = 4, 3
    gam = rng.standard_normal(npairs * (ncwo + 1)) * 2
    n = pnof.on_sigmoid(gam, npairs, ncwo)
    pair, _ = pnof.layout(npairs, ncwo)
    for g in range(npairs):
        assert abs(n[pair == g].sum() - 1.0) < 1e-15
    assert np.all((n > 0) & (n < 1))
    assert abs(2 * n.sum() - 2 * npairs) < 1e-13          # trace = number of electrons


def test_sigmoid_jacobian_fd():
    rng = np.random.default_rng(2)
    npairs, ncwo = 3, 2
    gam = rng.standard_normal(npairs * (ncwo + 1))
    jac = pnof.on_sigmoid_jac(gam, npairs, ncwo)
    h = 1e-6
    for r in range(len(gam)):
        e = np.zeros_like(gam)
        e[r] = h
        fd = (pnof.on_sigmoid(gam + e, npairs, ncwo) - pnof.on_sigmoid(gam - e, npairs, ncwo)) / (2 * h)
        assert np.max(np.abs(fd - jac[:, r])) < 1e-9


def test_sigmoid_equal_gammas_give_equal_shares():
    n = pnof.on_sigmoid(np.full(6, 0.3), 2, 2)
    assert np.allclose(n, 1.0 / 3.0, atol=1e-15)


# ------------------------------------------------------------------ trigonometric map
@pytest.mark.parametrize("npairs,ncwo", [(1, 1), (2, 3), (3, 4)])
def test_trig_sum_rules(npairs, ncwo):
    rng = np.random.default_rng(3)
    gam = rng.uniform(-3, 3, npairs * ncwo)
    n = pnof.on_trig(gam, npairs, ncwo)
    pair, strong = pnof.layout(npairs, ncwo)
    for g in range(npairs):
        assert abs(n[pair == g].sum() - 1.0) < 1e-15      # Eq. sum1 via Eqs. soo, woo
    assert np.all(n[strong[: len(n)]] >= 0.5) and np.all(n[strong[: len(n)]] <= 1.0)
    assert np.all(n[~strong[: len(n)]] <= 0.5) and np.all(n >= 0)


def test_trig_closed_forms():
    npairs, ncwo = 1, 2
    # gamma_g = 0: doubly occupied strong orbital, empty weak ones
    assert np.allclose(pnof.on_trig([0.0, 1.0], npairs, ncwo), [1.0, 0.0, 0.0], atol=1e-16)
    # gamma_g = pi/2: n_g = 1/2, hole 1/2; gamma_p1 = pi/4 splits the hole evenly
    n = pnof.on_trig([math.pi / 2, math.pi / 4], npairs, ncwo)
    assert np.allclose(n, [0.5, 0.25, 0.25], atol=1e-15)
    # single weak orbital takes the whole hole: n_w = sin^2(gamma)/2
    n = pnof.on_trig([0.7], 1, 1)
    assert abs(n[1] - 0.5 * math.sin(0.7) ** 2) < 1e-16


def test_trig_jacobian_fd():
    rng = np.random.default_rng(4)
    npairs, ncwo = 2, 4
    gam = rng.uniform(-2, 2, npairs * ncwo)
    jac = pnof.on_trig_jac(gam, npairs, ncwo)
    h = 1e-6
    for r in range(len(gam)):
        e = np.zeros_like(gam)
        e[r] = h
        fd = (pnof.on_trig(gam + e, npairs, ncwo) - pnof.on_trig(gam - e, npairs, ncwo)) / (2 * h)
        assert np.max(np.abs(fd - jac[:, r])) < 1e-9
