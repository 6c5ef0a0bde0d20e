"""Every launch-parameter choice the autotuner may make (chunk size, P-splits of the b and Y
contractions, the wide X and Y tile variants) gives the default plan's results within float32
summation-order differences, on shapes where the wide tiles leave ragged edges (nbf not a
multiple of 256)."""
import numpy as np
import pytest
import torch

import synth

P = pytest.importorskip("paper_2004_06142_amd")
pytestmark = pytest.mark.gpu

DEV = torch.device("cuda", 0)


def t(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to(DEV)


@pytest.fixture(scope="module")
def ctx():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    c = P.Context(0)
    yield c
    c.set_tuning(None)


TUNINGS = [
    dict(x_variant=1), dict(y_variant=1), dict(x_variant=1, y_variant=1),
    dict(pchunk=32), dict(pchunk=96, nsplit_b=3, nsplit_y=40), dict(nsplit_b=50, nsplit_y=2),
    dict(pchunk=40, nsplit_b=40, nsplit_y=40, y_variant=1),
]


@pytest.mark.parametrize("tuning", TUNINGS, ids=[str(x) for x in TUNINGS])
def test_tuning_choices_agree(ctx, tuning):
    inst = synth.make(synth.Workload("tune_300", 300, 1200, 30, 3, "bf16"), 9)
    wl = inst.wl
    prob = P.problem(wl.nbf, wl.naux, wl.npairs, wl.ncwo, P.PNOF7, P.BF16_SPLIT, P.INTS_DF_BF16)
    B = t(inst.B).to(torch.bfloat16)
    n = ctx.on_map(t(inst.gamma), wl.npairs, wl.ncwo)
    ctx.set_tuning(None)
    ref = ctx.lagrangian(prob, t(inst.C), n, t(inst.H), B, grads=True, jk=True)
    ctx.set_tuning(tuning)
    out = ctx.lagrangian(prob, t(inst.C), n, t(inst.H), B, grads=True, jk=True)
    torch.cuda.synchronize()
    ctx.set_tuning(None)
    assert abs(out["E"].item() - ref["E"].item()) < 1e-7
    for k, tol in (("lam", 1e-6), ("J", 1e-6), ("K", 1e-6), ("dEdC", 1e-5), ("dEdn", 1e-6)):
        assert torch.max(torch.abs(out[k] - ref[k])).item() < tol, k
