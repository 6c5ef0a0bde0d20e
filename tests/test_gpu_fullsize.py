"""Full-size parity on the configured workloads, in the launch configuration the benchmark times
(the autotuner's cached launch parameters for the shape when the cache holds them, as the benchmark
applies them; else the automatic plan).

Expected values are the oracle's, stored by tests/golden/make_expected.py (FP64, streamed route,
same seeded inputs): sampled entries in <name>_expected.json, and whole arrays in <name>_arrays.npz
-- at C3 every element of J, K, lambda, dE/dC (active columns), dE/dn and the orbital energies; at
C5 the diagonals of J and K, four whole rows and four whole active columns of lambda and dE/dC, all
of dE/dn and the orbital energies.  B is generated on the device by the seeded filler
(bit-identical to the host generator, see test_gpu_synth.py).  Energies: <= 1e-8 Ha (float64
path), <= 1e-6 Ha (bf16 split).
"""
import json
import os

import numpy as np
import pytest
import torch

import synth

P = pytest.importorskip("paper_2004_06142_amd")
from paper_2004_06142_amd import autotune  # noqa: E402

pytestmark = pytest.mark.gpu
GOLD = os.path.join(os.path.dirname(__file__), "golden")


def _load(name):
    path = os.path.join(GOLD, f"{name}_expected.json")
    if not os.path.exists(path):
        pytest.skip(f"{path} not generated")
    return json.load(open(path))


@pytest.fixture(scope="module")
def ctx():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return P.Context(0)


def _inputs(name):
    import synth.device as sdev
    inst = synth.workload(name, with_b=False)
    wl = inst.wl
    dev = torch.device("cuda", 0)
    t = lambda a: torch.from_numpy(np.ascontiguousarray(a)).to(dev)
    B = sdev.make_b(inst.key, wl.nbf, wl.naux, dtype=torch.bfloat16 if wl.b_dtype == "bf16" else torch.float64,
                    device=dev)
    kind = P.INTS_DF_BF16 if wl.b_dtype == "bf16" else P.INTS_DF_F64
    return inst, wl, t(inst.C), t(inst.H), t(inst.gamma), B, kind


def _sampled(out, ref, key, getter):
    got = np.array([getter(out, idx) for idx in ref[key]["idx"]])
    return np.max(np.abs(got - np.array(ref[key]["val"])))


def _arrays(name):
    path = os.path.join(GOLD, f"{name}_arrays.npz")
    return dict(np.load(path)) if os.path.exists(path) else None


def _array_errors(o, eps, arr, nact):
    """Max abs error over every stored element (whole matrices at C3, whole lines at C5)."""
    if "J" in arr:
        return {"J_all": np.max(np.abs(o["J"] - arr["J"])), "K_all": np.max(np.abs(o["K"] - arr["K"])),
                "lam_all": np.max(np.abs(o["lam"][:, :nact] - arr["lam"])),
                "lam_zero": np.max(np.abs(o["lam"][:, nact:])) if o["lam"].shape[1] > nact else 0.0,
                "dEdC_all": np.max(np.abs(o["dEdC"][:, :nact] - arr["dEdC"])),
                "dEdn_all": np.max(np.abs(o["dEdn"][:nact] - arr["dEdn"])),
                "eps_all": np.max(np.abs(eps - arr["eps"]))}
    rows, cols = arr["rows"], arr["cols"]
    return {"Jdiag": np.max(np.abs(np.diag(o["J"]) - arr["Jdiag"])),
            "Kdiag": np.max(np.abs(np.diag(o["K"]) - arr["Kdiag"])),
            "lam_lines": max(np.max(np.abs(o["lam"][rows, :nact] - arr["lam_rows"])),
                             np.max(np.abs(o["lam"][:, cols] - arr["lam_cols"]))),
            "dEdC_lines": max(np.max(np.abs(o["dEdC"][rows, :nact] - arr["dEdC_rows"])),
                              np.max(np.abs(o["dEdC"][:, cols] - arr["dEdC_cols"]))),
            "dEdn_all": np.max(np.abs(o["dEdn"][:nact] - arr["dEdn"])),
            "eps_all": np.max(np.abs(eps - arr["eps"]))}


@pytest.mark.parametrize("name", ["c3_df500", "c5_df1200"])
def test_full_size_parity(ctx, name):
    ref = _load(name)
    arr = _arrays(name)
    inst, wl, C, H, gam, B, kind = _inputs(name)
    res = {}
    for prec in (P.FP64, P.BF16_SPLIT):
        prob = P.problem(wl.nbf, wl.naux, wl.npairs, wl.ncwo, P.PNOF7, prec, kind)
        ent = autotune.apply_cached(ctx, prob)
        print(name, "prec", prec, "plan", ctx.plan(prob), "cached" if ent else "automatic")
        ctx.reserve(prob)
        n = ctx.on_map(gam, wl.npairs, wl.ncwo)
        out = ctx.lagrangian(prob, C, n, H, B, grads=True, jk=True)
        Cn, eps = ctx.orbital_step(out["lam"], C)
        o = {k: v.cpu().numpy() for k, v in out.items()}
        dE = abs(o["E"][0] - ref["E"])
        errs = {
            "E": dE,
            "J": _sampled(o, ref, "J", lambda d, i: d["J"][i[0], i[1]]),
            "K": _sampled(o, ref, "K", lambda d, i: d["K"][i[0], i[1]]),
            "lam": _sampled(o, ref, "lam", lambda d, i: d["lam"][i[0], i[1]]),
            "dEdC": _sampled(o, ref, "dEdC", lambda d, i: d["dEdC"][i[0], i[1]]),
            "dEdn": _sampled(o, ref, "dEdn", lambda d, i: d["dEdn"][i]),
            "eps": float(np.max(np.abs(eps.cpu().numpy() - np.array(ref["eps"])))),
            "max_asym": abs(o["max_asym"][0] - ref["max_asym"]),
        }
        if arr is not None:
            errs.update(_array_errors(o, eps.cpu().numpy(), arr, wl.nact))
        res[prec] = errs
        ctx.set_tuning(None)
        print(name, "prec", prec, {k: f"{v:.2e}" for k, v in errs.items()})
    e64, emx = res[P.FP64], res[P.BF16_SPLIT]
    assert e64["E"] < 1e-8 and e64["lam"] < 1e-10 and e64["J"] < 1e-12 and e64["K"] < 1e-12
    assert e64["dEdC"] < 1e-9 and e64["dEdn"] < 1e-9 and e64["eps"] < 1e-9
    assert emx["E"] < 1e-6 and emx["lam"] < 2e-5 and emx["J"] < 2e-5 and emx["K"] < 2e-5
    assert emx["eps"] < 2e-5 and emx["dEdC"] < 1e-4
    if arr is not None:
        lim64 = {"J_all": 1e-12, "K_all": 1e-12, "lam_all": 1e-10, "lam_zero": 0.0, "dEdC_all": 1e-9,
                 "dEdn_all": 1e-9, "eps_all": 1e-9, "Jdiag": 1e-12, "Kdiag": 1e-12, "lam_lines": 1e-10,
                 "dEdC_lines": 1e-9}
        limmx = {"J_all": 2e-5, "K_all": 2e-5, "lam_all": 2e-5, "lam_zero": 0.0, "dEdC_all": 1e-4,
                 "dEdn_all": 1e-4, "eps_all": 2e-5, "Jdiag": 2e-5, "Kdiag": 2e-5, "lam_lines": 2e-5,
                 "dEdC_lines": 1e-4}
        for k in lim64:
            if k in e64:
                assert e64[k] <= lim64[k], (k, e64[k])
                assert emx[k] <= limmx[k], (k, emx[k])


def test_finite_difference_gradients_c3(ctx):
    """dE/dC and dE/dgamma against central differences (h = 1e-5) of float64 energies, 32 entries each."""
    inst, wl, C, H, gam, B, kind = _inputs("c3_df500")
    p64 = P.problem(wl.nbf, wl.naux, wl.npairs, wl.ncwo, P.PNOF7, P.FP64, kind)
    pmx = P.problem(wl.nbf, wl.naux, wl.npairs, wl.ncwo, P.PNOF7, P.BF16_SPLIT, kind)
    g64 = P.energy_and_grad(ctx, p64, C, gam, H, B)
    gmx = P.energy_and_grad(ctx, pmx, C, gam, H, B)

    def energy(Cx, gx):
        n = ctx.on_map(gx, wl.npairs, wl.ncwo)
        return ctx.energy(p64, Cx, n, H, B).item()

    rng = np.random.default_rng(2004061422)
    h = 1e-5
    for _ in range(32):
        mu, q = int(rng.integers(0, wl.nbf)), int(rng.integers(0, wl.nact))
        Cp, Cm = C.clone(), C.clone()
        Cp[mu, q] += h
        Cm[mu, q] -= h
        fd = (energy(Cp, gam) - energy(Cm, gam)) / (2 * h)
        assert abs(fd - g64["dEdC"][mu, q].item()) < 1e-6 * max(1.0, abs(fd))
        assert abs(fd - gmx["dEdC"][mu, q].item()) < 1e-4 * max(1.0, abs(fd))
    for _ in range(32):
        r = int(rng.integers(0, wl.nact))
        gp, gm = gam.clone(), gam.clone()
        gp[r] += h
        gm[r] -= h
        fd = (energy(C, gp) - energy(C, gm)) / (2 * h)
        assert abs(fd - g64["dEdgamma"][r].item()) < 1e-6 * max(1.0, abs(fd))
        assert abs(fd - gmx["dEdgamma"][r].item()) < 1e-4 * max(1.0, abs(fd))
