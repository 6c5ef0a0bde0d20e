"""Every launch-parameter choice the autotuner may make (chunk size, P-splits of the b and Y
contractions, the wide X and Y tile variants) gives the default plan's results within float32
summation-order differences, on shapes where the wide tiles leave ragged edges (nbf not a
multiple of 256): nbf 300 (rows of B not 16-byte aligned, so X takes the register-staged form) and
nbf 552 with 276 active orbitals (aligned rows: every variant runs its direct-to-LDS form, and the
256-wide tiles cover the active orbitals in two tiles, the second ragged)."""
import numpy as np
import pytest
import torch

import synth
import synth.device as sdev

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


SHAPES = {
    "nbf300": synth.Workload("tune_300", 300, 1200, 30, 3, "bf16"),
    "nbf552": synth.Workload("tune_552", 552, 1104, 69, 3, "bf16"),
}
TUNINGS = [
    dict(x_variant=1, y_variant=1), dict(x_variant=2), dict(y_variant=2), dict(x_variant=2, y_variant=2),
    dict(y_variant=3), dict(y_variant=3, nsplit_y=7), dict(x_variant=3),
    dict(x_variant=3, y_variant=3, pchunk=40, nsplit_y=9),
    dict(pchunk=32), dict(pchunk=96, nsplit_b=3, nsplit_y=40), dict(nsplit_b=50, nsplit_y=2),
    dict(pchunk=40, nsplit_b=40, nsplit_y=40, y_variant=2),
]


_REF = {}


def _reference(ctx, shape):
    """Inputs of one shape (B made on the device by the bit-identical filler) and the default plan's
    outputs, computed once per shape."""
    if shape not in _REF:
        inst = synth.make(SHAPES[shape], 9, with_b=False)
        wl = inst.wl
        prob = P.problem(wl.nbf, wl.naux, wl.npairs, wl.ncwo, P.PNOF7, P.BF16_SPLIT, P.INTS_DF_BF16)
        B = sdev.make_b(inst.key, wl.nbf, wl.naux, dtype=torch.bfloat16, device=DEV)
        n = ctx.on_map(t(inst.gamma), wl.npairs, wl.ncwo)
        C, H = t(inst.C), t(inst.H)
        ctx.set_tuning(None)
        ref = ctx.lagrangian(prob, C, n, H, B, grads=True, jk=True)
        torch.cuda.synchronize()
        _REF[shape] = (prob, C, n, H, B, ref)
    return _REF[shape]


@pytest.mark.parametrize("shape", sorted(SHAPES))
@pytest.mark.parametrize("tuning", TUNINGS, ids=[str(x) for x in TUNINGS])
def test_tuning_choices_agree(ctx, tuning, shape):
    prob, C, n, H, B, ref = _reference(ctx, shape)
    ctx.set_tuning(tuning)
    out = ctx.lagrangian(prob, C, n, H, B, grads=True, jk=True)
    torch.cuda.synchronize()
    ctx.set_tuning(None)
    assert abs(out["E"].item() - ref["E"].item()) < 1e-7
    for k, tol in (("lam", 1e-6), ("J", 1e-6), ("K", 1e-6), ("dEdC", 1e-5), ("dEdn", 1e-6)):
        assert torch.max(torch.abs(out[k] - ref[k])).item() < tol, k
