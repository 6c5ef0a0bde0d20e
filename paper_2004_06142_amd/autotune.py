"""Launch-parameter autotuner for the density-fitted contractions.

For a problem shape it times candidate launch parameters (rows per chunk, P-splits of the b and Y
contractions, block-tile variants of X and Y) on the device with the library's own stage timers,
one stage at a time (coordinate search), and keeps the fastest.  Results are cached in a JSON file
keyed by GPU architecture, precision and a size bucket of (nbf, nact, naux); the path comes from
PNOF_AUTOTUNE_CACHE (default: autotune_cache.json next to this file).
"""
from __future__ import annotations

import json
import math
import os
import time

import torch

from . import Context, Tuning

CACHE = os.environ.get("PNOF_AUTOTUNE_CACHE",
                       os.path.join(os.path.dirname(os.path.abspath(__file__)), "autotune_cache.json"))


def _bucket(x: int) -> int:
    """Size bucket: powers of two split in quarters."""
    if x <= 0:
        return 0
    e = math.floor(math.log2(x))
    return int(2 ** e * (1 + math.floor(4 * (x / 2 ** e - 1)) / 4))


# bumped whenever the meaning of a tuning field changes, so stale entries are not applied
SCHEMA = 2


def key(prob, arch: str) -> str:
    return (f"v{SCHEMA}:{arch}:p{prob.precision}:i{prob.ints}:nbf{_bucket(prob.nbf)}:nact{_bucket(prob.nact)}"
            f":naux{_bucket(prob.naux)}")


def _arch(device) -> str:
    try:
        return torch.cuda.get_device_properties(device).gcnArchName.split(":")[0]
    except Exception:
        return "unknown"


def load_cache() -> dict:
    try:
        with open(CACHE) as f:
            return json.load(f)
    except (OSError, ValueError):
        return {}


def save_cache(c: dict):
    tmp = CACHE + ".tmp"
    with open(tmp, "w") as f:
        json.dump(c, f, indent=1, sort_keys=True)
    os.replace(tmp, CACHE)


def _time(ctx: Context, prob, run, reps: int) -> dict:
    run()                                    # warm (and size the workspace)
    torch.cuda.synchronize()
    ctx.profile_begin()
    t0 = time.perf_counter()
    for _ in range(reps):
        run()
    torch.cuda.synchronize()
    wall = (time.perf_counter() - t0) / reps
    st = ctx.profile_end()
    return {"wall": wall, **{k: v[0] / reps for k, v in st.items()}}


def apply_cached(ctx: Context, prob) -> dict | None:
    """Set the cached tuning of `prob` on `ctx` if the cache holds one (else leave the automatic plan);
    returns the entry or None."""
    ent = load_cache().get(key(prob, _arch(ctx.device)))
    ctx.set_tuning(ent["tuning"] if ent else None)
    return ent


def tune(ctx: Context, prob, run, reps: int = 2, use_cache: bool = True, verbose: bool = False) -> dict:
    """Pick launch parameters for `prob`; `run()` performs one library call on that problem."""
    arch = _arch(ctx.device)
    k = key(prob, arch)
    cache = load_cache() if use_cache else {}
    if k in cache:
        ctx.set_tuning(cache[k]["tuning"])
        return cache[k]
    ctx.set_tuning(None)
    base = ctx.plan(prob)
    best = dict(base)

    def measure(t):
        ctx.set_tuning(Tuning(**t))
        r = _time(ctx, prob, run, reps)
        if verbose:
            print("  tune", t, {a: round(b, 3) for a, b in r.items()}, flush=True)
        return r

    cur = measure(best)
    # chunk size first (it sets the scale of the other two splits)
    for pc in sorted({max(1, base["pchunk"] // 2), base["pchunk"], base["pchunk"] * 2}):
        if pc == best["pchunk"] or pc > prob.naux:
            continue
        t = dict(best, pchunk=pc, nsplit_b=0, nsplit_y=0)
        r = measure(t)
        if r["wall"] < cur["wall"]:
            best, cur = ctx.plan(prob), r
    ctx.set_tuning(Tuning(**best))
    # per-stage parameters, each judged on its own stage time; a Y tile variant is tried with the
    # P-split count the planner picks for it (the right count scales with the variant's tile count)
    for field, stage, cands in (("x_variant", "X", [1, 2, 3]), ("y_variant", "Y", [1, 2, 3])):
        for v in cands:
            if v == best[field]:
                continue
            trial = dict(best, **{field: v})
            if field == "y_variant":
                ctx.set_tuning(Tuning(**dict(trial, nsplit_y=0)))
                trial["nsplit_y"] = ctx.plan(prob)["nsplit_y"]
            r = measure(trial)
            if r[stage] < cur[stage] * 0.98:
                best, cur = trial, r
    for field, stage in (("nsplit_b", "b"), ("nsplit_y", "Y")):
        b0 = best[field]
        for v in (b0 // 2, b0 - 1, b0 + 1, b0 * 2):
            if v == best[field] or v < 1 or v > best["pchunk"]:
                continue
            r = measure(dict(best, **{field: v}))
            if r[stage] < cur[stage] * 0.98:
                best, cur = dict(best, **{field: v}), r
    ctx.set_tuning(Tuning(**best))
    entry = {"tuning": best, "ms": {a: 1e3 * b if a == "wall" else b for a, b in cur.items()}, "arch": arch,
             "shape": [prob.nbf, prob.nact, prob.naux]}
    if use_cache:
        cache = load_cache()
        cache[k] = entry
        save_cache(cache)
    return entry


def batch_key(batch, arch: str) -> str:
    """Cache key of a batch: its precision and the sorted (nbf, nact, naux) of its instances."""
    import hashlib
    shapes = sorted((p.nbf, p.nact, p.naux) for p in batch.problems)
    h = hashlib.sha1(repr(shapes).encode()).hexdigest()[:16]
    return f"v{SCHEMA}:{arch}:batch:p{batch.problems[0].precision}:n{len(shapes)}:{h}"


def tune_batch(batch, reps: int = 10, use_cache: bool = True, verbose: bool = False) -> dict:
    """Pick the tile widths (64 or 128 along the active orbitals) of a bound batch's grouped X, b and Y
    contractions by timing graph replays of the whole batch, one stage at a time from the automatic
    choice; the entry is cached under the batch's shape signature."""
    arch = _arch(batch.ctx.device)
    k = batch_key(batch, arch)
    cache = load_cache() if use_cache else {}
    if k in cache:
        batch.set_tiles(*cache[k]["tiles"])
        return cache[k]

    def measure(tiles):
        batch.set_tiles(*tiles)
        for _ in range(2):
            batch.run(graph=True)
        torch.cuda.synchronize()
        ts = []
        for _ in range(reps):
            a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            a.record()
            batch.run(graph=True)
            b.record()
            b.synchronize()
            ts.append(a.elapsed_time(b))
        ts.sort()
        ms = ts[len(ts) // 2]
        if verbose:
            print("  tune batch", tiles, round(ms, 3), flush=True)
        return ms

    batch.set_tiles(0, 0, 0)
    best = list(batch.tiles())
    cur = measure(best)
    for stage in range(3):
        trial = list(best)
        trial[stage] = 64 if best[stage] == 128 else 128
        ms = measure(trial)
        if ms < cur * 0.99:
            best, cur = trial, ms
    batch.set_tiles(*best)
    entry = {"tiles": best, "ms": cur, "arch": arch, "instances": len(batch.problems)}
    if use_cache:
        cache = load_cache()
        cache[k] = entry
        save_cache(cache)
    return entry


def main():
    """Tune one synthetic workload on device 0 and store the entry in the cache file."""
    import argparse

    import numpy as np

    import synth
    import synth.device as sdev

    from . import INTS_DF_BF16, INTS_DF_F64, PNOF7, BF16_SPLIT, FP64, problem

    ap = argparse.ArgumentParser()
    ap.add_argument("--workload", default="c5_df1200")
    ap.add_argument("--precision", default="bf16split", choices=["bf16split", "fp64"])
    ap.add_argument("--reps", type=int, default=2)
    args = ap.parse_args()
    dev = torch.device("cuda", 0)
    inst = synth.workload(args.workload, with_b=False)
    wl = inst.wl
    t = lambda a: torch.from_numpy(np.ascontiguousarray(a)).to(dev)
    C, H, gamma = t(inst.C), t(inst.H), t(inst.gamma)
    B = sdev.make_b(inst.key, wl.nbf, wl.naux, dtype=torch.bfloat16 if wl.b_dtype == "bf16" else torch.float64,
                    device=dev)
    kind = INTS_DF_BF16 if wl.b_dtype == "bf16" else INTS_DF_F64
    prec = BF16_SPLIT if args.precision == "bf16split" else FP64
    prob = problem(wl.nbf, wl.naux, wl.npairs, wl.ncwo, PNOF7, prec, kind)
    ctx = Context(0)
    ctx.reserve(prob)
    n = ctx.on_map(gamma, wl.npairs, wl.ncwo)
    ent = tune(ctx, prob, lambda: ctx.lagrangian(prob, C, n, H, B), reps=args.reps, use_cache=False, verbose=True)
    cache = load_cache()
    cache[key(prob, _arch(0))] = ent
    save_cache(cache)
    print(json.dumps(ent), flush=True)


if __name__ == "__main__":
    main()
