"""Write the oracle's expected values for the full-size workloads (runs on the CPU only).

Usage: python tests/golden/make_expected.py c5_df1200 [c3_df500] [pes64] ...
       python tests/golden/make_expected.py --arrays c3_df500 [c5_df1200]
Calls only ``oracle`` (FP64, streamed route) on inputs from ``synth``; B rows are regenerated
chunk by chunk from the counter-based stream, in worker processes, so that no full float64 copy of B
ever exists.  Output: tests/golden/<workload>_expected.json with the energy, the orbital-step
eigenvalues and sampled entries of J, K, lambda, dE/dC and dE/dn (indices stored with the values).
With --arrays: tests/golden/<workload>_arrays.npz instead, holding whole arrays -- at c3_df500 every
element of J, K, the active columns of lambda and dE/dC, dE/dn and the orbital energies; at
c5_df1200 the diagonals of J and K, LINES whole rows and whole active columns of lambda and dE/dC
(indices stored), dE/dn and the orbital energies.
"""
from __future__ import annotations

import json
import multiprocessing as mp
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import synth  # noqa: E402
from oracle import pnof, stream  # noqa: E402

CHUNK = 48


def _rows(args):
    key, nbf, naux, p0, p1, dt = args
    return p0, synth.b_chunk(key, nbf, naux, p0, p1, dt)


def oracle_run(name: str, workers: int = 6):
    """The streamed oracle's Lagrangian step and orbital energies on a named workload."""
    inst = synth.workload(name, with_b=False)
    wl = inst.wl
    n = pnof.on_sigmoid(inst.gamma, wl.npairs, wl.ncwo)
    ranges = [(inst.key, wl.nbf, wl.naux, p0, min(wl.naux, p0 + CHUNK), wl.b_dtype)
              for p0 in range(0, wl.naux, CHUNK)]
    t0 = time.time()
    with mp.get_context("fork").Pool(workers) as pool:
        it = pool.imap(_rows, ranges)
        pending = {}

        def chunk(p0, p1):
            while p0 not in pending:
                q0, rows = next(it)
                pending[q0] = rows
            rows = pending.pop(p0)
            assert rows.shape[0] == p1 - p0
            print(f"  rows {p0}..{p1} ({time.time() - t0:.0f} s)", flush=True)
            return rows

        r = stream.lagrangian(inst.C, n, inst.H, chunk, wl.npairs, wl.ncwo, pnof.PNOF7, naux=wl.naux,
                              pchunk=CHUNK)
    _, eps, _ = pnof.orbital_step(r["lam"], inst.C)
    return inst, wl, r, eps, time.time() - t0


LINES = 4


def arrays(name: str) -> dict:
    inst, wl, r, eps, sec = oracle_run(name)
    na = wl.nact
    if name == "c3_df500":
        return {"J": r["J"], "K": r["K"], "lam": r["lam"][:, :na], "dEdC": r["dEdC"][:, :na], "dEdn": r["dEdn"],
                "eps": eps, "E": np.array([r["E"]]), "seconds": np.array([sec])}
    rng = np.random.default_rng(23)
    rows = np.sort(rng.choice(wl.nbf, LINES, replace=False))
    cols = np.sort(rng.choice(na, LINES, replace=False))
    return {"Jdiag": np.diag(r["J"]).copy(), "Kdiag": np.diag(r["K"]).copy(), "rows": rows, "cols": cols,
            "lam_rows": r["lam"][rows, :na], "lam_cols": r["lam"][:, cols], "dEdC_rows": r["dEdC"][rows, :na],
            "dEdC_cols": r["dEdC"][:, cols], "dEdn": r["dEdn"], "eps": eps, "E": np.array([r["E"]]),
            "seconds": np.array([sec])}


def expected(name: str, workers: int = 6) -> dict:
    inst, wl, r, eps, sec = oracle_run(name, workers)
    t0 = time.time() - sec
    rng = np.random.default_rng(17)
    pq = rng.integers(0, wl.nact, size=(64, 2))
    lam_pq = np.stack([rng.integers(0, wl.nbf, 64), rng.integers(0, wl.nact, 64)], axis=1)
    mq = np.stack([rng.integers(0, wl.nbf, 32), rng.integers(0, wl.nact, 32)], axis=1)
    pn = rng.integers(0, wl.nact, 32)
    return {
        "workload": name, "seed": synth.seed_of(name), "functional": "PNOF7", "on_map": "sigmoid",
        "E": r["E"], "max_asym": pnof.max_asym(r["lam"]),
        "eps": eps.tolist(),
        "J": {"idx": pq.tolist(), "val": [r["J"][p, q] for p, q in pq]},
        "K": {"idx": pq.tolist(), "val": [r["K"][p, q] for p, q in pq]},
        "lam": {"idx": lam_pq.tolist(), "val": [r["lam"][p, q] for p, q in lam_pq]},
        "dEdC": {"idx": mq.tolist(), "val": [r["dEdC"][m, q] for m, q in mq]},
        "dEdn": {"idx": pn.tolist(), "val": [r["dEdn"][p] for p in pn]},
        "seconds": time.time() - t0,
    }


def _energy_term_scale(n, r, wl):
    """sqrt(sum (alpha J)^2 + (beta K)^2): the size of the two-electron energy terms."""
    alpha, beta = pnof.coefficients(n, wl.npairs, wl.ncwo, pnof.PNOF7)
    return float(np.sqrt(np.sum((alpha * r["J"]) ** 2) + np.sum((beta * r["K"]) ** 2)))


def expected_pes(ninst: int = 64) -> dict:
    """Every instance of the PES-scan batch (PNOF7, sigmoid ON map): E, max asymmetry and sampled
    lambda, dE/dC and dE/dn entries."""
    t0 = time.time()
    out = {"workload": "pes64", "seed": synth.seed_of("pes64"), "functional": "PNOF7", "on_map": "sigmoid",
           "instances": []}
    rng = np.random.default_rng(19)
    for i, inst in enumerate(synth.pes_scan(ninst, with_b=False)):
        wl = inst.wl
        B = synth.b_chunk(inst.key, wl.nbf, wl.naux, 0, wl.naux, wl.b_dtype)
        n = pnof.on_sigmoid(inst.gamma, wl.npairs, wl.ncwo)
        r = stream.lagrangian(inst.C, n, inst.H, B, wl.npairs, wl.ncwo, pnof.PNOF7)
        del B
        lam_pq = np.stack([rng.integers(0, wl.nbf, 16), rng.integers(0, wl.nact, 16)], axis=1)
        mq = np.stack([rng.integers(0, wl.nbf, 8), rng.integers(0, wl.nact, 8)], axis=1)
        pn = rng.integers(0, wl.nact, 8)
        out["instances"].append({
            "nbf": wl.nbf, "naux": wl.naux, "npairs": wl.npairs, "ncwo": wl.ncwo, "E": r["E"],
            "max_asym": pnof.max_asym(r["lam"]),
            "lam": {"idx": lam_pq.tolist(), "val": [r["lam"][p, q] for p, q in lam_pq]},
            "dEdC": {"idx": mq.tolist(), "val": [r["dEdC"][m, q] for m, q in mq]},
            "dEdn": {"idx": pn.tolist(), "val": [r["dEdn"][p] for p in pn]},
            "T": _energy_term_scale(n, r, wl),
        })
        print(f"  instance {i}: nbf {wl.nbf} E {r['E']:.10f} ({time.time() - t0:.0f} s)", flush=True)
    out["seconds"] = time.time() - t0
    return out


if __name__ == "__main__":
    if sys.argv[1] == "--arrays":
        for name in sys.argv[2:]:
            out = arrays(name)
            path = os.path.join(os.path.dirname(os.path.abspath(__file__)), f"{name}_arrays.npz")
            np.savez_compressed(path, **out)
            print(f"wrote {path} ({out['seconds'][0]:.0f} s)")
        sys.exit(0)
    for name in sys.argv[1:]:
        out = expected_pes() if name == "pes64" else expected(name)
        path = os.path.join(os.path.dirname(os.path.abspath(__file__)), f"{name}_expected.json")
        with open(path, "w") as f:
            json.dump(out, f)
        print(f"wrote {path} ({out['seconds']:.0f} s)")
