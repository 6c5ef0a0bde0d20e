"""Benchmark: PNOF7 energy + gradient iterations per second on one MI355X.

One step is the whole hot path on one batch of synthetic input:
  occupation map gamma -> n, Lagrangian (J, K, energy, Fock vectors, lambda, dE/dC, dE/dn,
  max asymmetry), ON-map adjoint dE/dgamma, and the orbital step (symmetrised lambda,
  float64 eigensolver, C_new = C U).
Default workload: N_bf = 1200, N_aux = 4800 (B in bfloat16, 13.8 GB, generated on the device),
100 pairs, 11 weak orbitals per pair (1200 active orbitals), bf16-split contractions.

Prints one JSON line (see the repository's measurement notes for the fields).
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK = {"bf16": 2.5e15, "f64": 78.6e12, "f32": 157.3e12}   # dense matrix-core peaks (bf16 = fp16)
KSRC = os.path.join(ROOT, "paper_2004_06142_amd", "csrc")
# HBM bytes per launch from the FETCH_SIZE and WRITE_SIZE counter runs (profiles/), each scaled by the
# factor a plain 1 GiB elementwise copy gives, and the SHA-256 of the kernel source they were taken on:
# once the source changes the figure no longer applies and traffic is reported as null.
TRAFFIC = {
    # profiles/c5_df1200_hbm_traffic.md: C5, bf16 split, 164-row chunks (read + written bytes per launch)
    ("gemm1_kernel", 3): {"bytes": 1616331062 + 926146614,
                          "plan": {"pchunk": 164, "x_variant": 3},
                          "sha256": {"k_gemm_bf16.hip": "739a0e927a9a5740758dc869d19722c729b4c658e67bcb213bd4cf4448b56ae8"}},
    ("gemm2_kernel", 3): {"bytes": 4146286647 + 639393009,
                          "plan": {"pchunk": 164, "nsplit_b": 18},
                          "sha256": {"k_gemm_bf16.hip": "739a0e927a9a5740758dc869d19722c729b4c658e67bcb213bd4cf4448b56ae8"}},
    ("gemm3_kernel", 3): {"bytes": 2586050632 + 57679787,
                          "plan": {"pchunk": 164, "nsplit_y": 10, "y_variant": 3},
                          "sha256": {"k_gemm_bf16.hip": "739a0e927a9a5740758dc869d19722c729b4c658e67bcb213bd4cf4448b56ae8"}},
}
GOLDEN_C5 = os.path.join(ROOT, "tests", "golden", "c5_df1200_expected.json")


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="c5_df1200")
    ap.add_argument("--precision", default="bf16split", choices=["bf16split", "fp64", "fp32", "bf16"])
    ap.add_argument("--fp64-steps", type=int, default=1, help="steps of the float64 path for the speedup (0: skip)")
    ap.add_argument("--cpu-rows", type=int, default=1024, help="rows of B in the oracle's timed sample (0: skip)")
    ap.add_argument("--pchunk", type=int, default=0)
    ap.add_argument("--no-tune", action="store_true", help="skip the launch-parameter autotuner")
    ap.add_argument("--pes-reps", type=int, default=20,
                    help="timed replays of the 64-instance PES-scan batch (0: skip that measurement)")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="MIB",
                    help="first run a plain device-to-device copy of this many MiB (reference for traffic counters)")
    ap.add_argument("--cpu-protocol", action="store_true",
                    help="instead of the benchmark: the host DGEMM rate and the float64 oracle timed on the host "
                         "cores (all threads and one thread) at C2 and C3, and over every row of B at C5")
    return ap.parse_args()


def stage_flops(wl, stage):
    """Algorithmic flops of one full pass of a contraction stage (one product per contraction)."""
    nb, na, nx = wl.nbf, wl.nact, wl.naux
    return {"X": 2.0 * nx * nb * nb * na, "b": 2.0 * nx * na * nb * na, "Y": 2.0 * nx * nb * na * na}[stage]


def _sha(path):
    import hashlib
    with open(path, "rb") as f:
        return hashlib.sha256(f.read()).hexdigest()


def traffic(kname, prec, plan):
    """Measured HBM bytes per launch of the dominant kernel, or None when no valid measurement exists."""
    ent = TRAFFIC.get((kname, prec))
    if not ent or ent["plan"] != {k: plan[k] for k in ent["plan"]}:
        return None
    if any(_sha(os.path.join(KSRC, f)) != h for f, h in ent["sha256"].items()):
        return None
    return ent["bytes"]


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only; --gpus {args.gpus} is not supported "
              "(sharding the auxiliary index across GPUs is described, not implemented).", file=sys.stderr)
        sys.exit(2)
    import numpy as np
    import torch

    import paper_2004_06142_amd as P
    import synth
    import synth.device as sdev

    dev = torch.device("cuda", 0)
    if args.cpu_protocol:
        print(json.dumps(cpu_protocol()), flush=True)
        return
    if args.copy_calibration:
        # one elementwise kernel that reads and writes exactly MIB MiB each (calibrates the HBM counters)
        src = torch.ones(args.copy_calibration << 18, dtype=torch.float32, device=dev)
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        torch.neg(src, out=dst)
        torch.cuda.synchronize()
        del src, dst
    wl = synth.WORKLOADS[args.workload]
    inst = synth.workload(args.workload, with_b=False)
    prec = {"bf16split": P.BF16_SPLIT, "fp64": P.FP64, "fp32": P.FP32, "bf16": P.BF16}[args.precision]
    t = lambda a: torch.from_numpy(np.ascontiguousarray(a)).to(dev)
    C0, H, gamma = t(inst.C), t(inst.H), t(inst.gamma)
    bdt = torch.bfloat16 if wl.b_dtype == "bf16" else torch.float64
    B = sdev.make_b(inst.key, wl.nbf, wl.naux, dtype=bdt, device=dev)
    kind = P.INTS_DF_BF16 if wl.b_dtype == "bf16" else P.INTS_DF_F64
    ctx = P.Context(0)
    if args.pchunk:
        ctx.set_pchunk(args.pchunk)

    def step(prob, C):
        out = P.energy_and_grad(ctx, prob, C, gamma, H, B)
        Cn, eps = ctx.orbital_step(out["lam"], C)
        return out, Cn

    def run(prob, warmup, steps, profile):
        ctx.reserve(prob)
        if not args.no_tune and not args.pchunk:
            from paper_2004_06142_amd import autotune
            n0 = ctx.on_map(gamma, prob.npairs, prob.ncwo)
            ent = autotune.tune(ctx, prob, lambda: ctx.lagrangian(prob, C0, n0, H, B), verbose=False)
            print(f"[bench] tuning {ent['tuning']}", file=sys.stderr, flush=True)
            ctx.reserve(prob)
        # the integrals stay fixed through an orbital optimisation: their row bounds (split mode) are
        # taken once, as a loop over iterations would, not in every step
        ctx.bind_integrals(prob, B)
        out = None
        for _ in range(warmup):
            out, _ = step(prob, C0)
        torch.cuda.synchronize()
        if profile:
            ctx.profile_begin()
        # HIP events around each step on the library's stream, for the median and p5 / p95
        evs = [torch.cuda.Event(enable_timing=True) for _ in range(steps + 1)]
        t0 = time.perf_counter()
        evs[0].record(ctx.stream)
        for i in range(steps):
            out, _ = step(prob, C0)
            evs[i + 1].record(ctx.stream)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        prof = ctx.profile_end() if profile else None
        per = np.array([evs[i].elapsed_time(evs[i + 1]) for i in range(steps)])
        return out, dt, prof, per

    prob = P.problem(wl.nbf, wl.naux, wl.npairs, wl.ncwo, P.PNOF7, prec, kind)
    print(f"[bench] workload {wl.name}: warmup {args.warmup}, timing {args.steps} steps", file=sys.stderr, flush=True)
    out, dt, prof, per = run(prob, args.warmup, args.steps, True)
    ms = 1e3 * dt / args.steps
    E = out["E"].item()
    print(f"[bench] {ms:.1f} ms/step, E = {E:.10f}, stages {prof}", file=sys.stderr, flush=True)

    # dominant contraction kernel and its roofline
    dtype_key = {P.FP64: "f64", P.FP32: "f32"}.get(prec, "bf16")
    stage = max(("X", "b", "Y"), key=lambda s: prof[s][0])
    st_ms, st_n = prof[stage]
    flops = stage_flops(wl, stage) * args.steps
    achieved = flops / (st_ms * 1e-3)
    terms = {"X": 2, "b": 3, "Y": 3}[stage] if prec == P.BF16_SPLIT else 1
    kname = {"X": "gemm1_kernel", "b": "gemm2_kernel", "Y": "gemm3_kernel"}[stage]
    roofline = {"bound": "mfma", "achieved": achieved / 1e12, "peak": PEAK[dtype_key] / 1e12, "unit": "TFLOP/s",
                "frac": achieved / PEAK[dtype_key], "traffic": traffic(kname, prec, ctx.plan(prob)),
                "kernel": kname,
                "avg_launch_ms": st_ms / st_n, "launches": st_n,
                "issued_frac": achieved * terms / PEAK[dtype_key]}
    stages = {k: {"ms_per_step": v[0] / args.steps, "launches_per_step": v[1] / args.steps} for k, v in prof.items()}

    result = {
        "metric": "PNOF7 energy+grad iterations/sec", "value": args.steps / dt, "unit": "iters/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup, "ms_per_step": ms, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None,
        "dtype": {"bf16split": "bf16+f16 (f32 acc, f64 sums)", "fp64": "f64", "fp32": "f32",
                  "bf16": "bf16 (f32 acc)"}[args.precision],
        "data": "synthetic",
        "config": {"workload": wl.name, "nbf": wl.nbf, "naux": wl.naux, "npairs": wl.npairs, "ncwo": wl.ncwo,
                   "nact": wl.nact, "functional": "PNOF7", "B": wl.b_dtype, "seed": synth.seed_of(wl.name),
                   "integrals": "bound once (pnof_bind_integrals): B's row bounds kept across steps"},
        "energy_Ha": E, "stages": stages, "roofline": roofline, "launch": ctx.plan(prob),
        "step_ms": {"median": float(np.median(per)), "p5": float(np.percentile(per, 5)),
                    "p95": float(np.percentile(per, 95)), "steps": int(len(per))},
    }
    if os.path.exists(GOLDEN_C5) and wl.name == "c5_df1200":
        ref = json.load(open(GOLDEN_C5))
        result["abs_err_Ha_vs_oracle"] = abs(E - ref["E"])
        # per-result error against the oracle's stored values (sampled entries, all orbital energies),
        # from one more call outside the timed region
        n0 = ctx.on_map(gamma, wl.npairs, wl.ncwo)
        o = ctx.lagrangian(prob, C0, n0, H, B, grads=True, jk=True)
        _, eps = ctx.orbital_step(o["lam"], C0)
        hv = {k: v.cpu().numpy() for k, v in o.items()}

        def worst(key, get):
            return float(max(abs(get(i) - v) for i, v in zip(ref[key]["idx"], ref[key]["val"])))

        result["errors_vs_oracle"] = {
            "E_Ha": float(abs(hv["E"][0] - ref["E"])),
            "J": worst("J", lambda i: hv["J"][i[0], i[1]]),
            "K": worst("K", lambda i: hv["K"][i[0], i[1]]),
            "lambda": worst("lam", lambda i: hv["lam"][i[0], i[1]]),
            "dEdC": worst("dEdC", lambda i: hv["dEdC"][i[0], i[1]]),
            "dEdn": worst("dEdn", lambda i: hv["dEdn"][i]),
            "eps": float(np.max(np.abs(eps.cpu().numpy() - np.array(ref["eps"])))),
            "max_asym": float(abs(hv["max_asym"][0] - ref["max_asym"])),
            "note": "max abs error over the sampled entries ("
                    + ", ".join(f"{k} {len(ref[k]['idx'])}" for k in ("J", "K", "lam", "dEdC", "dEdn"))
                    + f") and all {len(ref['eps'])} orbital energies",
        }

    if args.fp64_steps > 0 and prec != P.FP64:
        p64 = P.problem(wl.nbf, wl.naux, wl.npairs, wl.ncwo, P.PNOF7, P.FP64, kind)
        print("[bench] float64 path for the speedup", file=sys.stderr, flush=True)
        o64, dt64, prof64, _ = run(p64, 0, args.fp64_steps, True)
        result["fp64_path"] = {"ms_per_step": 1e3 * dt64 / args.fp64_steps, "energy_Ha": o64["E"].item(),
                               "speedup_of_mixed": (dt64 / args.fp64_steps) / (dt / args.steps),
                               "abs_dE_mixed_vs_fp64": abs(E - o64["E"].item()),
                               "stages_ms": {k: v[0] / args.fp64_steps for k, v in prof64.items()}}
    del B
    torch.cuda.empty_cache()

    if args.pes_reps > 0:
        result["pes_batch"] = pes_batch(P, ctx, args.pes_reps, tune=not args.no_tune)
        torch.cuda.empty_cache()

    if args.cpu_rows > 0:
        result["cpu_baseline"] = cpu_baseline(wl, inst, args.cpu_rows)
    print(json.dumps(result), flush=True)


GOLDEN_PES = os.path.join(ROOT, "tests", "golden", "pes64_expected.json")


def pes_batch(P, ctx, reps, tune=True):
    """The 64-instance PES scan (N_bf in [40, 300], bf16 split) as one graph-replayed batch, in both
    forms (the grouped launch sequence and the persistent launch); the faster one heads the record."""
    import numpy as np
    import torch

    import synth
    import synth.device as sdev

    dev = ctx.device
    insts = synth.pes_scan(64, with_b=False)
    probs, ins = [], []
    for inst in insts:
        wl = inst.wl
        probs.append(P.problem(wl.nbf, wl.naux, wl.npairs, wl.ncwo, P.PNOF7, P.BF16_SPLIT, P.INTS_DF_BF16))
        t = lambda a: torch.from_numpy(np.ascontiguousarray(a)).to(dev)
        ins.append({"C": t(inst.C), "H": t(inst.H), "n": ctx.on_map(t(inst.gamma), wl.npairs, wl.ncwo),
                    "B": sdev.make_b(inst.key, wl.nbf, wl.naux, dtype=torch.bfloat16, device=dev)})
    batch = P.Batch(ctx, probs)
    outs = batch.bind(ins)
    if tune:
        from paper_2004_06142_amd import autotune
        autotune.tune_batch(batch)

    def timed(persistent):
        for _ in range(3):
            batch.run(graph=True, persistent=persistent)
        torch.cuda.synchronize()
        ms, done = [], []
        for _ in range(reps):
            a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            a.record()
            batch.run(graph=True, persistent=persistent)
            b.record()
            b.synchronize()
            ms.append(a.elapsed_time(b))
            if persistent:
                done.append(batch.times())
        return np.array(ms), (np.array(done) if persistent else None)

    flops = sum(2.0 * p.naux * p.nbf * p.nact * (p.nbf + 2 * p.nact) for p in probs)

    def summary(ms, launches):
        med = float(np.median(ms))
        return {"ms_per_batch_p50": med, "ms_p90": float(np.percentile(ms, 90)),
                "ms_p99": float(np.percentile(ms, 99)), "instances_per_s": len(probs) / (med * 1e-3),
                "launches_per_batch": launches, "algorithmic_tflops": flops / (med * 1e-3) / 1e12}

    seq = summary(timed(False)[0], batch.info()["launches"])
    seq["note"] = "every instance completes with the batch's last grouped launch: per-instance latency = batch latency"
    pms, done = timed(True)
    per = summary(pms, 2)
    # per-instance completion times (device clock, from the run's start) over all instances x timed runs
    samples = np.asarray(done).ravel()
    per["instance_latency_ms"] = {"p50": float(np.percentile(samples, 50)) * 1e-3,
                                  "p90": float(np.percentile(samples, 90)) * 1e-3,
                                  "p99": float(np.percentile(samples, 99)) * 1e-3,
                                  "max": float(samples.max()) * 1e-3, "samples": int(samples.size)}
    best = "persistent" if per["ms_per_batch_p50"] < seq["ms_per_batch_p50"] else "launch_sequence"
    head = per if best == "persistent" else seq
    res = {"instances": len(probs), "nbf_range": [min(p.nbf for p in probs), max(p.nbf for p in probs)],
           "tiles_xby": list(batch.tiles()), "graph": True, "mode": best,
           **{k: head[k] for k in ("ms_per_batch_p50", "ms_p90", "ms_p99", "instances_per_s", "algorithmic_tflops")},
           "persistent": per, "launch_sequence": seq}
    batch.run(graph=True, persistent=best == "persistent")
    torch.cuda.synchronize()
    if os.path.exists(GOLDEN_PES):
        ref = json.load(open(GOLDEN_PES))
        res["max_abs_dE_vs_oracle"] = max(abs(o["E"].item() - r["E"]) for o, r in zip(outs, ref["instances"]))
    batch.close()
    return res


def cpu_baseline(wl, inst, rows):
    """The FP64 oracle (streamed route) timed on a bounded sample of the same workload."""
    import numpy as np
    import torch

    import synth.device as sdev
    from oracle import pnof, stream

    try:
        from threadpoolctl import threadpool_info
        cores = max([i.get("num_threads", 1) for i in threadpool_info() if i.get("internal_api") == "openblas"] or [1])
    except Exception:
        cores = os.cpu_count()
    rows = min(rows, wl.naux)
    out = torch.empty((rows, wl.nbf, wl.nbf), dtype=torch.bfloat16 if wl.b_dtype == "bf16" else torch.float64,
                      device="cuda")
    sdev.fill_b(out, inst.key, wl.nbf, wl.naux, 0)
    Bs = out.to(torch.float64).cpu().numpy()
    del out
    n = pnof.on_sigmoid(inst.gamma, wl.npairs, wl.ncwo)
    print(f"[bench] cpu oracle on {rows} of {wl.naux} rows of B", file=sys.stderr, flush=True)
    t0 = time.perf_counter()
    stream.lagrangian(inst.C, n, inst.H, Bs[:0], wl.npairs, wl.ncwo, pnof.PNOF7, naux=0)
    t_fixed = time.perf_counter() - t0
    t0 = time.perf_counter()
    r = stream.lagrangian(inst.C, n, inst.H, Bs, wl.npairs, wl.ncwo, pnof.PNOF7, naux=rows)
    t_rows = time.perf_counter() - t0
    t0 = time.perf_counter()
    pnof.orbital_step(r["lam"], inst.C)
    t_orb = time.perf_counter() - t0
    per_row = max(0.0, t_rows - t_fixed) / rows
    s_iter = t_fixed + per_row * wl.naux + t_orb
    return {"value": 1.0 / s_iter, "unit": "iters/s", "cores": cores, "kind": "oracle",
            "sample": f"streamed FP64 oracle over {rows} of {wl.naux} B rows ({t_rows:.1f} s), per-row cost scaled "
                      f"to all rows, plus its fixed part ({t_fixed:.1f} s) and orbital step ({t_orb:.1f} s)",
            "seconds_per_iter_est": s_iter}


def cpu_protocol():
    """The float64 oracle on the host cores: DGEMM rate, then one energy + lambda + gradient step (+ the
    orbital step's eigensolver at C1, C2, C3 and C5) per configuration, timed with every OpenBLAS
    thread, with 8 and with one (C5: every thread).  B
    is drawn before the clock starts (at C5 on the device, 96 rows at a time, widened to float64 and
    copied to the host; only the oracle's work on each chunk is timed, every row of B is used)."""
    import numpy as np
    import torch
    from threadpoolctl import threadpool_info, threadpool_limits

    import synth
    import synth.device as sdev
    from oracle import pnof, stream

    nthr = max([i.get("num_threads", 1) for i in threadpool_info() if i.get("internal_api") == "openblas"] or [1])
    res = {"host_threads": nthr, "cpu_count": os.cpu_count()}

    def dgemm_rate(n=4096, reps=3):
        a = np.random.default_rng(0).standard_normal((n, n))
        b = a.T.copy()
        a @ b
        ts = []
        for _ in range(reps):
            t0 = time.perf_counter()
            a @ b
            ts.append(time.perf_counter() - t0)
        return 2.0 * n ** 3 / min(ts) / 1e9

    res["dgemm_gflops"] = dgemm_rate()
    with threadpool_limits(8, user_api="blas"):
        res["dgemm_gflops_8threads"] = dgemm_rate()
    with threadpool_limits(1, user_api="blas"):
        res["dgemm_gflops_1thread"] = dgemm_rate(2048)

    # C1: the explicit-integral path (generalised Fock matrix from the 24^4 tensor, energy, lambda,
    # orbital step), median of 5
    inst = synth.workload("c1_eri24")
    w = inst.wl
    n = pnof.on_sigmoid(inst.gamma, w.npairs, w.ncwo)

    def c1():
        t0 = time.perf_counter()
        F = pnof.fock_ao(inst.C, n, inst.H, inst.ERI, w.npairs, w.ncwo, pnof.PNOF7, kind="eri")
        pnof.energy(inst.C, n, inst.H, inst.ERI, w.npairs, w.ncwo, pnof.PNOF7, kind="eri")
        pnof.orbital_step(pnof.lagrangian(inst.C, F), inst.C)
        return time.perf_counter() - t0

    res["c1_eri24"] = {"seconds_all_threads": float(np.median([c1() for _ in range(5)])), "runs": 5}
    with threadpool_limits(1, user_api="blas"):
        res["c1_eri24"]["seconds_1thread"] = float(np.median([c1() for _ in range(5)]))

    def step(inst, n, B, naux):
        t0 = time.perf_counter()
        r = stream.lagrangian(inst.C, n, inst.H, B, inst.wl.npairs, inst.wl.ncwo, pnof.PNOF7, naux=naux)
        pnof.orbital_step(r["lam"], inst.C)
        return time.perf_counter() - t0

    for name, reps in (("c2_df200", 5), ("c3_df500", 3)):
        inst = synth.workload(name, with_b=False)
        w = inst.wl
        bdt = torch.bfloat16 if w.b_dtype == "bf16" else torch.float64
        B = sdev.make_b(inst.key, w.nbf, w.naux, dtype=bdt, device=torch.device("cuda", 0)).to(torch.float64).cpu().numpy()
        n = pnof.on_sigmoid(inst.gamma, w.npairs, w.ncwo)
        ent = {"seconds_all_threads": float(np.median([step(inst, n, B, None) for _ in range(reps)]))}
        with threadpool_limits(8, user_api="blas"):
            ent["seconds_8threads"] = float(np.median([step(inst, n, B, None) for _ in range(reps)]))
        with threadpool_limits(1, user_api="blas"):
            ent["seconds_1thread"] = step(inst, n, B, None)
        del B
        ent["runs"] = reps
        res[name] = ent
        del inst
        print(f"[cpu] {name}: {ent}", file=sys.stderr, flush=True)

    # C4: the 64-instance PES scan, one Lagrangian + gradient per instance (B drawn before each clock)
    c4 = {"seconds_all_threads": 0.0, "seconds_8threads": 0.0, "seconds_1thread": 0.0, "instances": 64}
    for inst in synth.pes_scan(64, with_b=False):
        w = inst.wl
        B = synth.b_chunk(inst.key, w.nbf, w.naux, 0, w.naux, w.b_dtype).astype(np.float64)
        n = pnof.on_sigmoid(inst.gamma, w.npairs, w.ncwo)
        for key, lim in (("seconds_all_threads", None), ("seconds_8threads", 8), ("seconds_1thread", 1)):
            with threadpool_limits(lim, user_api="blas"):
                t0 = time.perf_counter()
                stream.lagrangian(inst.C, n, inst.H, B, w.npairs, w.ncwo, pnof.PNOF7)
                c4[key] += time.perf_counter() - t0
        del B
    res["c4_pes64"] = c4
    print(f"[cpu] c4_pes64: {c4}", file=sys.stderr, flush=True)

    wl = synth.WORKLOADS["c5_df1200"]
    inst = synth.workload("c5_df1200", with_b=False)
    n = pnof.on_sigmoid(inst.gamma, wl.npairs, wl.ncwo)
    rows = 96
    dev = torch.device("cuda", 0)
    buf = torch.empty((rows, wl.nbf, wl.nbf), dtype=torch.bfloat16, device=dev)
    gen = [0.0]

    def chunk(p0, p1):
        # drawing the rows and moving them to the host is not the oracle's work: its time is subtracted
        t0 = time.perf_counter()
        sdev.fill_b(buf[:p1 - p0], inst.key, wl.nbf, wl.naux, p0)
        host = buf[:p1 - p0].to(torch.float64).cpu().numpy()
        gen[0] += time.perf_counter() - t0
        if p0 % (8 * rows) == 0:
            print(f"[cpu] c5_df1200 rows {p0}..{p1} of {wl.naux}", file=sys.stderr, flush=True)
        return host

    t0 = time.perf_counter()
    r = stream.lagrangian(inst.C, n, inst.H, chunk, wl.npairs, wl.ncwo, pnof.PNOF7, naux=wl.naux, pchunk=rows)
    t_wall = time.perf_counter() - t0
    t1 = time.perf_counter()
    pnof.orbital_step(r["lam"], inst.C)
    t_orb = time.perf_counter() - t1
    t_total = t_wall - gen[0]
    res["c5_df1200"] = {"seconds_lagrangian": t_total, "seconds_orbital_step": t_orb,
                        "seconds_per_iter": t_total + t_orb, "rows": wl.naux, "chunk_rows": rows,
                        "seconds_drawing_rows": gen[0]}
    print(f"[cpu] c5_df1200: {res['c5_df1200']}", file=sys.stderr, flush=True)
    return res


if __name__ == "__main__":
    main()
