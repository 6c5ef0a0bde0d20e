"""NOF-MP2 reference terms (pnof_nofmp2_terms, Eqs. HFL and Esta) through the C ABI against the
oracle.  Float64: 1e-10 Ha.  bf16 split: E_hf and E_sta are plain sums of J and K, which carry the
2^-17 rounding of the split orbitals C~ to first order (the energy removes that term with its
first-order correction 4 <Y, C - C~>; these sums have no Fock vectors of their own to do the same),
so the bound is 2^-17 times the root-sum-square of their terms, sqrt(sum (2J - K)^2 + K^2), or
1e-6 Ha if larger."""
import numpy as np
import pytest
import torch

import synth
from oracle import pnof

P = pytest.importorskip("paper_2004_06142_amd")
pytestmark = pytest.mark.gpu

DEV = torch.device("cuda", 0)


def t(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to(DEV)


@pytest.fixture(scope="module")
def ctx():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return P.Context(0)


@pytest.mark.parametrize("name,prec,kind,tol", [
    ("c1_eri24", P.FP64, P.INTS_ERI4_F64, 1e-10),
    ("c2_df200", P.FP64, P.INTS_DF_F64, 1e-10),
    ("c2_df200", P.BF16_SPLIT, P.INTS_DF_F64, None),
])
def test_nofmp2_terms_match_oracle(ctx, name, prec, kind, tol):
    inst = synth.workload(name)
    wl = inst.wl
    n = pnof.on_sigmoid(inst.gamma, wl.npairs, wl.ncwo)
    naux = 0 if kind == P.INTS_ERI4_F64 else wl.naux
    prob = P.problem(wl.nbf, naux, wl.npairs, wl.ncwo, P.PNOF7, prec, kind)
    ints = t(inst.ERI) if kind == P.INTS_ERI4_F64 else t(inst.B)
    e_hf, e_sta = ctx.nofmp2_terms(prob, t(inst.C), t(n), t(inst.H), ints)
    J, K = pnof.jk_no(inst.ERI if kind == P.INTS_ERI4_F64 else inst.B, inst.C, wl.nact,
                      "eri" if kind == P.INTS_ERI4_F64 else "df")
    r_hf, r_sta = pnof.nofmp2_reference(n, pnof.h_no(inst.C, inst.H, wl.nact), J, K, wl.npairs, wl.ncwo)
    if tol is None:
        g = wl.npairs
        tol = max(1e-6, 2.0 ** -17 * np.sqrt(np.sum((2 * J[:g, :g] - K[:g, :g]) ** 2) + np.sum(K ** 2)))
    print(f"{name} prec={prec}: dE_hf={abs(e_hf.item() - r_hf):.2e} dE_sta={abs(e_sta.item() - r_sta):.2e} tol={tol:.1e}")
    assert abs(e_hf.item() - r_hf) < tol
    assert abs(e_sta.item() - r_sta) < tol


def test_nofmp2_hartree_fock_limit(ctx):
    inst = synth.workload("c1_eri24")
    wl = inst.wl
    n = np.zeros(wl.nact)
    n[:wl.npairs] = 1.0
    prob = P.problem(wl.nbf, 0, wl.npairs, wl.ncwo, P.PNOF7, P.FP64, P.INTS_ERI4_F64)
    e_hf, e_sta = ctx.nofmp2_terms(prob, t(inst.C), t(n), t(inst.H), t(inst.ERI))
    E = ctx.energy(prob, t(inst.C), t(n), t(inst.H), t(inst.ERI))
    assert e_sta.item() == 0.0
    assert abs(e_hf.item() - E.item()) < 1e-10


def test_repeated_driver_calls_allocate_nothing(ctx):
    """The driver calls keep their device buffers in the context: after a first call, repeating it
    (and the occupation optimiser) leaves the device's free memory unchanged."""
    inst = synth.workload("c2_df200")
    wl = inst.wl
    n = pnof.on_sigmoid(inst.gamma, wl.npairs, wl.ncwo)
    prob = P.problem(wl.nbf, wl.naux, wl.npairs, wl.ncwo, P.PNOF7, P.FP64, P.INTS_DF_F64)
    C, nn, H, B = t(inst.C), t(n), t(inst.H), t(inst.B)
    first = ctx.nofmp2_terms(prob, C, nn, H, B)
    again = ctx.nofmp2_terms(prob, C, nn, H, B)   # torch's pool now holds the outputs' blocks too
    torch.cuda.synchronize()
    free0 = torch.cuda.mem_get_info(DEV)[0]
    for _ in range(3):
        again = ctx.nofmp2_terms(prob, C, nn, H, B)
        torch.cuda.synchronize()
        assert again[0].item() == first[0].item() and again[1].item() == first[1].item()
    assert torch.cuda.mem_get_info(DEV)[0] == free0
