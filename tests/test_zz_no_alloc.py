"""pnof_lagrangian_noalloc (workspace in the library's static device array, nothing allocated)
through the C ABI against pnof_lagrangian on the same inputs, two calls in a row with the second
on a smaller problem, and against the oracle.  Bars: float64 path 1e-10 Ha and lambda 1e-10 between
the two entry points (they differ only in the rows of B per chunk and the float64 GEMM), 1e-8 Ha to
the oracle; bf16 split 1e-6 Ha and lambda 2e-5, to each other and to the oracle."""
import ctypes

import numpy as np
import pytest
import torch

import synth
from oracle import pnof, stream

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


def _noalloc(ctx, prob, C, n, H, B):
    f = P.lib().pnof_lagrangian_noalloc
    nbf, nact = prob.nbf, prob.nact
    z = lambda *s: torch.zeros(*s, dtype=torch.float64, device=DEV)
    out = {"lam": z(nbf, nbf), "E": z(1), "dEdC": z(nbf, nbf), "dEdn": z(nact), "max_asym": z(1), "J": z(nact, nact),
           "K": z(nact, nact)}
    p = lambda x: ctypes.c_void_p(x.data_ptr())
    st = f(ctx.handle, ctypes.byref(prob), p(C), p(n), p(H), p(B), p(out["lam"]), p(out["E"]), p(out["dEdC"]),
           p(out["dEdn"]), p(out["max_asym"]), p(out["J"]), p(out["K"]))
    return st, out


CASES = [   # the second call is the smaller problem
    ("c2_df200", 200, 800, 20, 4, "f64", P.BF16_SPLIT),
    ("small", 96, 160, 6, 3, "bf16", P.FP64),
    ("small_split", 72, 130, 5, 3, "bf16", P.BF16_SPLIT),
]


def test_noalloc_matches_lagrangian_twice(ctx):
    for name, nbf, naux, npairs, ncwo, bdt, prec in CASES:
        inst = synth.make(synth.Workload(name, nbf, naux, npairs, ncwo, bdt), 3)
        n = pnof.on_sigmoid(inst.gamma, npairs, ncwo)
        kind = P.INTS_DF_F64 if bdt == "f64" else P.INTS_DF_BF16
        B = t(inst.B) if bdt == "f64" else t(inst.B).to(torch.bfloat16)
        prob = P.problem(nbf, naux, npairs, ncwo, P.PNOF7, prec, kind)
        C, nd, H = t(inst.C), t(n), t(inst.H)
        st, out = _noalloc(ctx, prob, C, nd, H, B)
        assert st == 0, P.lib().pnof_last_error(ctx.handle)
        ref = ctx.lagrangian(prob, C, nd, H, B, grads=True, jk=True)
        torch.cuda.synchronize()
        orc = stream.lagrangian(inst.C, n, inst.H, inst.B, npairs, ncwo, pnof.PNOF7)
        e_tol, l_tol = (1e-10, 1e-10) if prec == P.FP64 else (1e-6, 2e-5)
        d = {k: torch.max(torch.abs(out[k] - ref[k])).item() for k in ("E", "lam", "dEdC", "dEdn", "J", "K", "max_asym")}
        dE_oracle = abs(out["E"].item() - orc["E"])
        print(name, prec, {k: f"{v:.2e}" for k, v in d.items()}, f"oracle dE {dE_oracle:.2e}")
        assert d["E"] < e_tol and d["lam"] < l_tol and d["J"] < l_tol and d["K"] < l_tol
        assert d["dEdC"] < 10 * l_tol and d["dEdn"] < 10 * l_tol and d["max_asym"] < l_tol
        assert dE_oracle < (1e-8 if prec == P.FP64 else 1e-6)
        assert np.max(np.abs(out["lam"].cpu().numpy() - orc["lam"])) < (1e-10 if prec == P.FP64 else 2e-5)


def test_noalloc_rejects_a_problem_beyond_the_static_workspace(ctx):
    """Rejected on the host, before anything is enqueued: the inputs are never read."""
    prob = P.problem(2048, 4, 200, 9, P.PNOF7, P.FP64, P.INTS_DF_F64)
    dummy = torch.zeros(8, dtype=torch.float64, device=DEV)
    f = P.lib().pnof_lagrangian_noalloc
    p = ctypes.c_void_p(dummy.data_ptr())
    st = f(ctx.handle, ctypes.byref(prob), p, p, p, p, p, p, None, None, None, None, None)
    assert st == 7   # PNOF_E_UNSUPPORTED
    assert b"bytes of workspace" in P.lib().pnof_last_error(ctx.handle)
