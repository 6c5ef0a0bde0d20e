"""Small seeded systems for the CPU oracle pins (inputs from ``synth`` only)."""
from __future__ import annotations

import numpy as np

import synth


def system(nbf, naux, npairs, ncwo, seed=7, dtype="f64"):
    wl = synth.Workload(f"small_{nbf}_{naux}_{npairs}_{ncwo}", nbf, naux, npairs, ncwo, dtype)
    inst = synth.make(wl, seed)
    # boost the integral scale so that two-electron terms are not negligible in small tests
    return inst


def sigmoid_n(inst):
    from oracle import pnof
    wl = inst.wl
    return pnof.on_sigmoid(inst.gamma, wl.npairs, wl.ncwo)


def eri(inst):
    from oracle import pnof
    return pnof.eri_from_df(inst.B)


def rng(seed=0):
    return np.random.default_rng(seed)
