"""Multiplets (N_I singly occupied orbitals, Section 2) through the C ABI against the oracle.

Float64 path: |dE| <= 1e-8 Ha, lambda 1e-10; bf16 split: the single-problem mixed tolerances.
Also the restricted open-shell limit of PNOF7 against the high-spin determinant energy, the ON
maps with singles, the NOF-MP2 reference terms, the orbital loop and a batch with singles.
"""
import numpy as np
import pytest
import torch

import synth
from oracle import optimize as oopt
from oracle import pnof, stream
from tests import _brute

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


def _case(nbf, naux, npairs, ncwo, nsingle, dtype="f64", seed=41):
    inst = synth.make(synth.Workload(f"mult_{nbf}_{nsingle}", nbf, naux, npairs, ncwo, dtype), seed)
    nact = npairs * (ncwo + 1) + nsingle
    gamma = np.random.default_rng(seed).standard_normal(nact)
    return inst, gamma, nact


@pytest.mark.parametrize("func", [P.PNOF7, P.PNOF5, P.PNOF7S])
@pytest.mark.parametrize("prec,bdt", [(P.FP64, "f64"), (P.FP32, "f64"), (P.BF16_SPLIT, "bf16")])
def test_lagrangian_with_singles_matches_oracle(ctx, func, prec, bdt):
    npairs, ncwo, ns = 4, 3, 3
    inst, gamma, nact = _case(72, 288, npairs, ncwo, ns, bdt)
    n = pnof.on_sigmoid(gamma, npairs, ncwo, ns)
    kind = P.INTS_DF_F64 if bdt == "f64" else P.INTS_DF_BF16
    B = t(inst.B) if bdt == "f64" else t(inst.B).to(torch.bfloat16)
    prob = P.problem(72, 288, npairs, ncwo, func, prec, kind, nsingle=ns)
    nd = ctx.on_map(t(gamma), npairs, ncwo, nsingle=ns)
    assert np.max(np.abs(nd.cpu().numpy() - n)) < 1e-15
    out = ctx.lagrangian(prob, t(inst.C), nd, t(inst.H), B, grads=True, jk=True)
    r = stream.lagrangian(inst.C, n, inst.H, inst.B, npairs, ncwo, func, nsingle=ns)
    E = out["E"].item()
    if prec == P.FP64:
        assert abs(E - r["E"]) < 1e-8
        assert np.max(np.abs(out["lam"].cpu().numpy() - r["lam"])) < 1e-10
        assert np.max(np.abs(out["dEdn"].cpu().numpy() - r["dEdn"])) < 1e-9
        assert np.max(np.abs(out["dEdC"].cpu().numpy() - r["dEdC"])) < 1e-9
    else:
        assert abs(E - r["E"]) < 1e-6
        assert np.max(np.abs(out["lam"].cpu().numpy() - r["lam"])) < 2e-5
        assert np.max(np.abs(out["dEdC"].cpu().numpy() - r["dEdC"])) < 1e-4


@pytest.mark.parametrize("func,npairs,ns,prec", [(P.PNOF7, 43, 5, P.BF16_SPLIT), (P.PNOF5, 43, 5, P.BF16_SPLIT),
                                                  (P.PNOF7S, 44, 0, P.BF16_SPLIT), (P.PNOF7, 44, 0, P.BF16_SPLIT),
                                                  (P.PNOF7, 43, 5, P.FP32)])
def test_large_active_space_split_mode(ctx, func, npairs, ns, prec):
    """Active spaces past 512 orbitals in the bf16 split mode: the symmetric W (the transposed image
    of b's lower-triangle tiles) and Y's block-wise reads over many 128-blocks; nact = 521 and 528
    leave ragged tails of 128 and 256, and singles give one-orbital subspaces (beta_pp = 0).  The
    float32 mode on the same shape, at the same tolerances."""
    nbf, naux, ncwo = 560, 240, 11
    inst, gamma, nact = _case(nbf, naux, npairs, ncwo, ns, "bf16", seed=43)
    assert nact >= 512 and nact % 128 != 0
    n = pnof.on_sigmoid(gamma, npairs, ncwo, ns)
    prob = P.problem(nbf, naux, npairs, ncwo, func, prec, P.INTS_DF_BF16, nsingle=ns)
    out = ctx.lagrangian(prob, t(inst.C), t(n), t(inst.H), t(inst.B).to(torch.bfloat16), grads=True, jk=True)
    r = stream.lagrangian(inst.C, n, inst.H, inst.B, npairs, ncwo, func, nsingle=ns)
    o = {k: v.cpu().numpy() for k, v in out.items()}
    jk_tol = max(2e-5, 2.0 ** -14 * max(np.max(np.abs(r["J"])), np.max(np.abs(r["K"]))))
    errs = {"E": abs(o["E"][0] - r["E"]), "lam": np.max(np.abs(o["lam"] - r["lam"])),
            "dEdC": np.max(np.abs(o["dEdC"] - r["dEdC"])), "J": np.max(np.abs(o["J"] - r["J"])),
            "K": np.max(np.abs(o["K"] - r["K"])), "dEdn": np.max(np.abs(o["dEdn"][:nact] - r["dEdn"]))}
    print(func, nact, {k: f"{v:.2e}" for k, v in errs.items()})
    assert errs["E"] < 1e-6 and errs["lam"] < 2e-5 and errs["dEdC"] < 1e-4
    assert errs["J"] < jk_tol and errs["K"] < jk_tol and errs["dEdn"] < 1e-4


@pytest.mark.parametrize("kind", [P.ON_SIGMOID, P.ON_TRIG])
def test_on_map_and_adjoint_with_singles(ctx, kind):
    npairs, ncwo, ns = 3, 2, 2
    nact = npairs * (ncwo + 1) + ns
    rng = np.random.default_rng(6)
    ngam = nact if kind == P.ON_SIGMOID else npairs * ncwo
    gamma = rng.standard_normal(ngam)
    n, jac = ctx.on_map(t(gamma), npairs, ncwo, kind, jacobian=True, nsingle=ns)
    okind = "sigmoid" if kind == P.ON_SIGMOID else "trig"
    assert np.max(np.abs(n.cpu().numpy() - oopt.on_map(gamma, npairs, ncwo, okind, ns))) < 1e-15
    assert np.max(np.abs(jac.cpu().numpy() - oopt.on_jac(gamma, npairs, ncwo, okind, ns))) < 1e-14
    dEdn = rng.standard_normal(nact)
    g = ctx.on_map_vjp(t(gamma), t(dEdn), npairs, ncwo, kind, nsingle=ns)
    assert np.max(np.abs(g.cpu().numpy() - oopt.on_jac(gamma, npairs, ncwo, okind, ns).T @ dEdn)) < 1e-13


def test_restricted_open_shell_limit_on_device(ctx):
    inst = synth.workload("c1_eri24")
    npairs, ncwo, ns = 3, 1, 2
    nact = npairs * (ncwo + 1) + ns
    n = np.zeros(nact)
    n[:npairs] = 1.0
    n[npairs:npairs + ns] = 0.5
    prob = P.problem(24, 0, npairs, ncwo, P.PNOF7, P.FP64, P.INTS_ERI4_F64, nsingle=ns)
    E = ctx.energy(prob, t(inst.C), t(n), t(inst.H), t(inst.ERI)).item()
    closed = list(range(npairs))
    E_det = _brute.determinant_energy(inst.C, inst.H, inst.ERI, closed + list(range(npairs, npairs + ns)), closed)
    assert abs(E - E_det) < 1e-9


def test_nofmp2_terms_with_singles(ctx):
    npairs, ncwo, ns = 4, 3, 2
    inst, gamma, nact = _case(64, 256, npairs, ncwo, ns)
    n = pnof.on_sigmoid(gamma, npairs, ncwo, ns)
    prob = P.problem(64, 256, npairs, ncwo, P.PNOF7, P.FP64, P.INTS_DF_F64, nsingle=ns)
    e_hf, e_sta = ctx.nofmp2_terms(prob, t(inst.C), t(n), t(inst.H), t(inst.B))
    J, K = pnof.jk_no(inst.B, inst.C, nact, "df")
    r_hf, r_sta = pnof.nofmp2_reference(n, pnof.h_no(inst.C, inst.H, nact), J, K, npairs, ncwo, ns)
    assert abs(e_hf.item() - r_hf) < 1e-10 and abs(e_sta.item() - r_sta) < 1e-10


def test_orbital_loop_with_singles_matches_oracle(ctx):
    npairs, ncwo, ns = 2, 1, 2
    inst, gamma, nact = _case(10, 40, npairs, ncwo, ns, seed=43)
    C0 = np.linalg.eigh(inst.H)[1]
    prob = P.problem(10, 40, npairs, ncwo, P.PNOF7, P.FP64, P.INTS_DF_F64, nsingle=ns)
    r = ctx.optimize(prob, t(inst.H), t(inst.B), t(C0), gamma=t(gamma), maxit=10, ndiis=4, delta=0.0,
                     on_gtol=1e-11)
    o = oopt.optimize(C0, gamma, inst.H, inst.B, npairs, ncwo, maxit=10, ndiis=4, delta=0.0, eps_n=0, eps_phi=0,
                      eps=0, nsingle=ns)
    assert r["iterations"] == o["iterations"] == 10
    assert abs(r["E"] - o["E"]) < 1e-8
    assert np.all(r["n"].cpu().numpy()[npairs:npairs + ns] == 0.5)


def test_batch_with_singles(ctx):
    import synth.device as sdev
    sizes = [(48, 2, 1), (96, 1, 2), (64, 3, 0)]
    probs, ins, refs = [], [], []
    for i, (nbf, ns, seed) in enumerate(sizes):
        npairs, ncwo = nbf // 10, 3
        inst, gamma, nact = _case(nbf, 4 * nbf, npairs, ncwo, ns, "bf16", seed=50 + i)
        n = pnof.on_sigmoid(gamma, npairs, ncwo, ns)
        probs.append(P.problem(nbf, 4 * nbf, npairs, ncwo, P.PNOF7, P.BF16_SPLIT, P.INTS_DF_BF16, nsingle=ns))
        B = sdev.make_b(inst.key, nbf, 4 * nbf, dtype=torch.bfloat16, device=DEV)
        ins.append({"C": t(inst.C), "H": t(inst.H), "n": t(n), "B": B, "gamma": t(gamma)})
        r = stream.lagrangian(inst.C, n, inst.H, inst.B, npairs, ncwo, P.PNOF7, nsingle=ns)
        r["dEdgamma"] = pnof.on_sigmoid_jac(gamma, npairs, ncwo, ns).T @ r["dEdn"]
        refs.append((r, n, npairs, ncwo, ns))
    batch = P.Batch(ctx, probs)
    outs = batch.bind(ins)
    # the grouped launch sequence and the persistent form (dE/dgamma through the ON map with singles)
    for persistent in (False, True):
        for o in outs:
            for v in o.values():
                v.fill_(float("nan"))
        batch.run(graph=True, persistent=persistent)
        torch.cuda.synchronize()
        if persistent:
            assert len(batch.times()) == len(probs)
        for o, (r, n, npairs, ncwo, ns) in zip(outs, refs):
            assert abs(o["E"].item() - r["E"]) < 1e-6, persistent
            assert np.max(np.abs(o["lam"].cpu().numpy() - r["lam"])) < 2e-5
            assert np.max(np.abs(o["dEdn"].cpu().numpy() - r["dEdn"])) < 2e-5
            assert np.max(np.abs(o["dEdgamma"].cpu().numpy() - r["dEdgamma"])) < 5e-5
