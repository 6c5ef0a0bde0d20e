"""Batched PES scan (pnof_batch_*) through the C ABI against the FP64 oracle.

Small batches are compared element by element with the oracle (streamed route) on the same
seeded inputs; the full 64-instance scan (N_bf integer-uniform in [40, 300], N_aux = 4 N_bf,
N_bf/10 pairs, 3 weak orbitals each, bf16 B) against stored oracle values
(tests/golden/pes64_expected.json).  Tolerances are those of the single-problem bf16-split path:
|dE| <= 1e-6 Ha, lambda / dE/dn to 2e-5, dE/dC to 1e-4.
"""
import json
import os

import numpy as np
import pytest
import torch

import synth
from oracle import pnof, stream

P = pytest.importorskip("paper_2004_06142_amd")
pytestmark = pytest.mark.gpu

DEV = torch.device("cuda", 0)
GOLD = os.path.join(os.path.dirname(__file__), "golden", "pes64_expected.json")


def t(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to(DEV)


@pytest.fixture(scope="module")
def ctx():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return P.Context(0)


def _device_inputs(ctx, inst, with_host_b=True):
    import synth.device as sdev
    wl = inst.wl
    B = sdev.make_b(inst.key, wl.nbf, wl.naux, dtype=torch.bfloat16, device=DEV)
    gam = t(inst.gamma)
    n = ctx.on_map(gam, wl.npairs, wl.ncwo)
    return {"C": t(inst.C), "H": t(inst.H), "n": n, "B": B}


def _small_batch(ninst=6, lo=40, hi=150, seed=2004061425):
    return synth.pes_scan(ninst, seed=seed, nbf_range=(lo, hi), with_b=True)


FUNCS = [P.PNOF7, P.PNOF5, P.PNOF7S]


@pytest.mark.parametrize("prec", [P.BF16_SPLIT, P.BF16])
def test_batch_matches_oracle(ctx, prec):
    insts = _small_batch()
    funcs = [FUNCS[i % 3] for i in range(len(insts))]
    probs = [P.problem(i.wl.nbf, i.wl.naux, i.wl.npairs, i.wl.ncwo, f, prec, P.INTS_DF_BF16)
             for i, f in zip(insts, funcs)]
    batch = P.Batch(ctx, probs)
    ins = [_device_inputs(ctx, i) for i in insts]
    outs = batch.bind(ins)
    batch.run(graph=False)
    torch.cuda.synchronize()
    for inst, func, o in zip(insts, funcs, outs):
        wl = inst.wl
        n = pnof.on_sigmoid(inst.gamma, wl.npairs, wl.ncwo)
        r = stream.lagrangian(inst.C, n, inst.H, inst.B, wl.npairs, wl.ncwo, func)
        E = o["E"].item()
        lam = o["lam"].cpu().numpy()
        if prec == P.BF16_SPLIT:
            assert abs(E - r["E"]) < 1e-6, (wl.nbf, E, r["E"])
            assert np.max(np.abs(lam - r["lam"])) < 2e-5
            assert np.max(np.abs(o["dEdC"].cpu().numpy() - r["dEdC"])) < 1e-4
            assert np.max(np.abs(o["dEdn"].cpu().numpy() - r["dEdn"])) < 2e-5
            assert abs(o["max_asym"].item() - pnof.max_asym(r["lam"])) < 2e-5
        else:
            # one bf16 product per contraction: an error study, bounded far more loosely
            scale = max(1.0, abs(r["E"]))
            assert abs(E - r["E"]) < 2e-2 * scale
            assert np.max(np.abs(lam - r["lam"])) < 5e-2 * max(1.0, np.max(np.abs(r["lam"])))
        # inactive columns are exactly zero
        assert np.all(lam[:, wl.nact:] == 0.0)


def test_batch_equals_single_problem_path(ctx):
    """Each instance of a batch against the single-problem entry point on the same inputs.  The two
    group the rows of B differently into float32 partial sums, so they agree to the mixed-precision
    tolerances, not bit for bit."""
    insts = _small_batch(4, 60, 200, seed=2004061426)
    probs = [P.problem(i.wl.nbf, i.wl.naux, i.wl.npairs, i.wl.ncwo, P.PNOF7, P.BF16_SPLIT, P.INTS_DF_BF16)
             for i in insts]
    batch = P.Batch(ctx, probs)
    ins = [_device_inputs(ctx, i) for i in insts]
    outs = batch.bind(ins)
    batch.run(graph=True)
    torch.cuda.synchronize()
    for prob, x, o in zip(probs, ins, outs):
        ref = ctx.lagrangian(prob, x["C"], x["n"], x["H"], x["B"], grads=True)
        torch.cuda.synchronize()
        assert abs(o["E"].item() - ref["E"].item()) < 1e-6
        assert torch.max(torch.abs(o["lam"] - ref["lam"])).item() < 2e-5
        assert torch.max(torch.abs(o["dEdn"] - ref["dEdn"])).item() < 2e-5
        assert torch.max(torch.abs(o["dEdC"] - ref["dEdC"])).item() < 1e-4


def test_batch_tiny_instances(ctx):
    """Instances far below one tile (N_bf 10..13, two active orbitals): fewer energy terms than the
    32 blocks that sum them per instance, one partial lower-triangle tile, padded rows of B.  Each
    against the single-problem entry point, on a graph replay and again on a second replay (the
    asymmetry maximum is cleared and raised anew on every run)."""
    insts = synth.pes_scan(4, seed=2004061427, nbf_range=(10, 13), ncwo=1, with_b=True)
    probs = [P.problem(i.wl.nbf, i.wl.naux, i.wl.npairs, i.wl.ncwo, P.PNOF7, P.BF16_SPLIT, P.INTS_DF_BF16)
             for i in insts]
    assert all(i.wl.npairs * (i.wl.ncwo + 1) == 2 for i in insts)
    batch = P.Batch(ctx, probs)
    ins = [_device_inputs(ctx, i) for i in insts]
    outs = batch.bind(ins)
    for _ in range(2):
        batch.run(graph=True)
        torch.cuda.synchronize()
        for prob, x, o in zip(probs, ins, outs):
            ref = ctx.lagrangian(prob, x["C"], x["n"], x["H"], x["B"], grads=True)
            torch.cuda.synchronize()
            assert abs(o["E"].item() - ref["E"].item()) < 1e-6
            assert torch.max(torch.abs(o["lam"] - ref["lam"])).item() < 2e-5
            assert torch.max(torch.abs(o["dEdn"] - ref["dEdn"])).item() < 2e-5
            assert torch.max(torch.abs(o["dEdC"] - ref["dEdC"])).item() < 1e-4
            assert abs(o["max_asym"].item() - ref["max_asym"].item()) < 2e-5
    batch.close()


def test_graph_replays_match_eager(ctx):
    """Graph replays, with eager library work and synchronisations between them, reproduce the
    eager result bit for bit (the same kernels in the same order)."""
    insts = _small_batch(5, 40, 160, seed=2004061427)
    probs = [P.problem(i.wl.nbf, i.wl.naux, i.wl.npairs, i.wl.ncwo, P.PNOF7, P.BF16_SPLIT, P.INTS_DF_BF16)
             for i in insts]
    batch = P.Batch(ctx, probs)
    ins = [_device_inputs(ctx, i) for i in insts]
    outs = batch.bind(ins)
    batch.run(graph=False)
    torch.cuda.synchronize()
    ref = [{k: v.clone() for k, v in o.items()} for o in outs]
    for rep in range(4):
        for o in outs:
            for v in o.values():
                v.fill_(float("nan"))
        batch.run(graph=True)
        torch.cuda.synchronize()
        for o, r in zip(outs, ref):
            for k in r:
                assert torch.equal(o[k], r[k]), (rep, k)
        # unrelated eager work on the same stream between replays
        p0 = probs[0]
        ctx.lagrangian(p0, ins[0]["C"], ins[0]["n"], ins[0]["H"], ins[0]["B"], grads=True)
        torch.cuda.synchronize()


def test_rebind_with_new_orbitals(ctx):
    """Binding new inputs (a rotated C) refreshes the results and discards the old graph."""
    insts = _small_batch(3, 40, 120, seed=2004061428)
    probs = [P.problem(i.wl.nbf, i.wl.naux, i.wl.npairs, i.wl.ncwo, P.PNOF7, P.BF16_SPLIT, P.INTS_DF_BF16)
             for i in insts]
    batch = P.Batch(ctx, probs)
    ins = [_device_inputs(ctx, i) for i in insts]
    batch.bind(ins)
    batch.run(graph=True)
    torch.cuda.synchronize()
    rng = np.random.default_rng(3)
    ins2 = []
    for inst, x in zip(insts, ins):
        Q, _ = np.linalg.qr(rng.standard_normal((inst.wl.nbf, inst.wl.nbf)))
        ins2.append(dict(x, C=t(inst.C @ Q)))
    outs = batch.bind(ins2)
    batch.run(graph=True)
    torch.cuda.synchronize()
    for inst, x, o in zip(insts, ins2, outs):
        wl = inst.wl
        n = pnof.on_sigmoid(inst.gamma, wl.npairs, wl.ncwo)
        r = stream.lagrangian(x["C"].cpu().numpy(), n, inst.H, inst.B, wl.npairs, wl.ncwo, pnof.PNOF7)
        assert abs(o["E"].item() - r["E"]) < 1e-6


# tile widths along the active orbitals of the grouped X, b, Y (None: the automatic choice); the
# 64-wide forms cut the padding of the short active spaces (nact = 0.4 nbf in [16, 120])
TILES = [None, (128, 128, 128), (64, 64, 64), (64, 128, 64), (128, 64, 128)]


@pytest.mark.parametrize("tiles", TILES, ids=[str(t) for t in TILES])
def test_full_pes_scan_against_stored_oracle_values(ctx, tiles):
    if not os.path.exists(GOLD):
        pytest.skip("pes64 expected values not generated")
    ref = json.load(open(GOLD))
    insts = synth.pes_scan(64, with_b=False)
    probs = [P.problem(i.wl.nbf, i.wl.naux, i.wl.npairs, i.wl.ncwo, P.PNOF7, P.BF16_SPLIT, P.INTS_DF_BF16)
             for i in insts]
    batch = P.Batch(ctx, probs)
    ins = [_device_inputs(ctx, i) for i in insts]
    outs = batch.bind(ins)
    if tiles is not None:
        batch.set_tiles(*tiles)        # after bind: offsets recomputed, graph dropped
        assert batch.tiles() == tiles
    batch.run(graph=True)
    torch.cuda.synchronize()
    worst = {"E": 0.0, "lam": 0.0, "dEdC": 0.0, "dEdn": 0.0}
    for inst, o, r in zip(insts, outs, ref["instances"]):
        assert inst.wl.nbf == r["nbf"]
        dE = abs(o["E"].item() - r["E"])
        assert dE < 1e-6, (inst.wl.nbf, dE)
        lam = o["lam"].cpu().numpy()
        dC = o["dEdC"].cpu().numpy()
        dn = o["dEdn"].cpu().numpy()
        el = max(abs(lam[p, q] - v) for (p, q), v in zip(r["lam"]["idx"], r["lam"]["val"]))
        ec = max(abs(dC[m, q] - v) for (m, q), v in zip(r["dEdC"]["idx"], r["dEdC"]["val"]))
        en = max(abs(dn[p] - v) for p, v in zip(r["dEdn"]["idx"], r["dEdn"]["val"]))
        assert el < 2e-5 and ec < 1e-4 and en < 2e-5, (inst.wl.nbf, el, ec, en)
        assert abs(o["max_asym"].item() - r["max_asym"]) < 2e-5
        for k, v in (("E", dE), ("lam", el), ("dEdC", ec), ("dEdn", en)):
            worst[k] = max(worst[k], v)
    print("pes64 worst errors", batch.tiles(), {k: f"{v:.2e}" for k, v in worst.items()})
    batch.close()


def test_batch_tile_tuner(ctx):
    """The batch autotuner times the tile widths of a bound batch and leaves a valid choice in place;
    results under every choice agree with the 128-wide reference to float32 summation order."""
    from paper_2004_06142_amd import autotune
    insts = synth.pes_scan(6, seed=11, with_b=False)
    probs = [P.problem(i.wl.nbf, i.wl.naux, i.wl.npairs, i.wl.ncwo, P.PNOF7, P.BF16_SPLIT, P.INTS_DF_BF16)
             for i in insts]
    batch = P.Batch(ctx, probs)
    outs = batch.bind([_device_inputs(ctx, i) for i in insts])
    batch.set_tiles(128, 128, 128)
    batch.run(graph=False)
    torch.cuda.synchronize()
    ref = [float(o["E"].item()) for o in outs]
    ent = autotune.tune_batch(batch, reps=3, use_cache=False)
    assert tuple(ent["tiles"]) == batch.tiles() and all(t in (64, 128) for t in ent["tiles"])
    batch.run(graph=True)
    torch.cuda.synchronize()
    for o, e in zip(outs, ref):
        assert abs(o["E"].item() - e) < 1e-7
    with pytest.raises(P.PnofError, match="PNOF_E_ARG"):
        batch.set_tiles(96, 0, 0)
    batch.close()


def test_batch_error_paths(ctx):
    good = P.problem(64, 256, 6, 3, P.PNOF7, P.BF16_SPLIT, P.INTS_DF_BF16)
    with pytest.raises(P.PnofError, match="PNOF_E_UNSUPPORTED"):
        P.Batch(ctx, [P.problem(64, 256, 6, 3, P.PNOF7, P.FP64, P.INTS_DF_BF16)])
    with pytest.raises(P.PnofError, match="PNOF_E_UNSUPPORTED"):
        P.Batch(ctx, [P.problem(64, 256, 6, 3, P.PNOF7, P.BF16_SPLIT, P.INTS_DF_F64)])
    with pytest.raises(P.PnofError, match="PNOF_E_ARG"):
        P.Batch(ctx, [good, P.problem(64, 256, 6, 3, P.PNOF7, P.BF16, P.INTS_DF_BF16)])
    with pytest.raises(P.PnofError, match="PNOF_E_SHAPE"):
        P.Batch(ctx, [good, P.problem(20, 80, 6, 3, P.PNOF7, P.BF16_SPLIT, P.INTS_DF_BF16)])
    b = P.Batch(ctx, [good])
    with pytest.raises(P.PnofError, match="PNOF_E_ARG"):
        b.run()
    assert b.info()["launches"] == 16   # 14 (the last forms dE/dgamma) + the two of the split mode's scale bounds
