"""Seeded synthetic inputs for the PNOF orbital-optimisation hot path.

This module holds none of the method's arithmetic.  It only draws the inputs
that the device library and the CPU oracle both consume:

* ``H``      symmetric one-electron matrix, off-diagonal N(0,1), diagonal -U(5,20);
* ``C``      orthogonal orbital coefficients, the Q factor of a Gaussian matrix;
* ``gamma``  one N(0,1) auxiliary variable per active orbital;
* ``B``      the density-fitting factor B[P, mu, nu], symmetric in (mu, nu), with
             B = exp(-|mu-nu|/6) / sqrt(naux) * G and G "Gaussian";
* ``ERI``    for the explicit-integral workload, (mu nu|la si) = sum_P B B.

H, C and gamma come from ``numpy.random.default_rng`` on the host.  B can be
tens of GB, so it comes from a counter-based stream that the host (numpy, here)
and the device (``synth/csrc/synth_fill.hip``) evaluate bit-identically:

* generator: SplitMix64 (Steele, Lea & Flood, OOPSLA 2014; output mixer of
  Vigna's reference code): draw(key, c) = mix64(key + (c+1) * 0x9E3779B97F4A7C15);
* normal deviate: Irwin-Hall sum of twelve 16-bit uniforms, centred; it has
  mean 0, variance 1 - 2^-32 and support [-6, 6], and uses integer arithmetic
  only, so both sides produce the same double exactly;
* element (P, i, j), i <= j, takes draws 3*((P*nbf + i)*nbf + j) + {0,1,2}; the
  (j, i) element reuses the (i, j) draws, so B_P is exactly symmetric;
* the decay/scale factor table f[k] = exp(-k/6)/sqrt(naux) is evaluated once
  here in float64 and handed to the device, so value = f[|i-j|] * g is one
  correctly rounded product on both sides;
* bfloat16 storage rounds that float64 value to nearest-even directly (no
  float32 intermediate), including the bf16 subnormal range.

The ERI workload builds its explicit tensor from a float64 B.
"""
from __future__ import annotations

import dataclasses
import math
from typing import Optional

import numpy as np

BASE_SEED = 2004061420
_GOLDEN = np.uint64(0x9E3779B97F4A7C15)
_M1 = np.uint64(0xBF58476D1CE4E5B9)
_M2 = np.uint64(0x94D049BB133111EB)
_IH_CENTRE = 393210  # 12 * 32767.5


@dataclasses.dataclass(frozen=True)
class Workload:
    """Shape of one PNOF problem (all sizes are per instance)."""

    name: str
    nbf: int
    naux: int          # density-fitting rank (the ERI workload also uses it to build ERI)
    npairs: int
    ncwo: int
    b_dtype: str       # "f64" or "bf16": storage type of B
    eri4: bool = False # explicit 4-index integrals are the input instead of B
    functional: int = 7

    @property
    def nact(self) -> int:
        return self.npairs * (self.ncwo + 1)


# The five workloads the hot path is measured on.
WORKLOADS = {
    "c1_eri24": Workload("c1_eri24", 24, 96, 5, 1, "f64", eri4=True),
    "c2_df200": Workload("c2_df200", 200, 800, 20, 4, "f64"),
    "c3_df500": Workload("c3_df500", 500, 2000, 50, 5, "bf16"),
    "c5_df1200": Workload("c5_df1200", 1200, 4800, 100, 11, "bf16"),
}
WORKLOAD_INDEX = {"c1_eri24": 0, "c2_df200": 1, "c3_df500": 2, "pes64": 3, "c5_df1200": 4}


def seed_of(name: str) -> int:
    return BASE_SEED + WORKLOAD_INDEX[name]


# ---------------------------------------------------------------- counter-based stream
def mix64(z: np.ndarray) -> np.ndarray:
    """SplitMix64 output mixer on uint64 arrays (wrapping arithmetic)."""
    z = np.asarray(z, dtype=np.uint64)
    with np.errstate(over="ignore"):
        z = (z ^ (z >> np.uint64(30))) * _M1
        z = (z ^ (z >> np.uint64(27))) * _M2
    return z ^ (z >> np.uint64(31))


def stream_key(seed: int, stream: int = 0) -> int:
    """64-bit key of an independent stream (one per B tensor / instance)."""
    s = np.uint64((seed * 0x100000001B3 + stream * 0xD1B54A32D192ED03) & 0xFFFFFFFFFFFFFFFF)
    return int(mix64(np.array([s], dtype=np.uint64))[0])


def draws(key: int, ctr: np.ndarray) -> np.ndarray:
    ctr = np.asarray(ctr, dtype=np.uint64)
    with np.errstate(over="ignore"):
        return mix64(np.uint64(key) + (ctr + np.uint64(1)) * _GOLDEN)


def ih12(key: int, idx: np.ndarray) -> np.ndarray:
    """Irwin-Hall(12) normal deviates for element indices ``idx`` (float64, exact)."""
    idx = np.asarray(idx, dtype=np.uint64)
    s = np.zeros(idx.shape, dtype=np.int64)
    base = idx * np.uint64(3)
    m16 = np.uint64(0xFFFF)
    for t in range(3):
        d = draws(key, base + np.uint64(t))
        for sh in (0, 16, 32, 48):
            s += ((d >> np.uint64(sh)) & m16).astype(np.int64)
    return (s - _IH_CENTRE).astype(np.float64) / 65536.0


def b_factor_table(nbf: int, naux: int) -> np.ndarray:
    """f[k] = exp(-k/6)/sqrt(naux), k = |mu-nu|; shared verbatim with the device fill."""
    k = np.arange(nbf, dtype=np.float64)
    return np.exp(-k / 6.0) / math.sqrt(naux)


def bf16_round(x: np.ndarray) -> np.ndarray:
    """Round float64 to the nearest bfloat16 (ties to even); returns float64 values."""
    x = np.asarray(x, dtype=np.float64)
    out = x.copy()                        # zeros keep their sign
    nz = x != 0.0
    _, e = np.frexp(x[nz])                # x = m 2^e, 0.5 <= |m| < 1 -> floor(log2|x|) = e-1
    qe = np.maximum(e - 1, -126) - 7
    out[nz] = np.rint(x[nz] * np.ldexp(1.0, -qe)) * np.ldexp(1.0, qe)
    return out


def f64_to_bf16_bits(x: np.ndarray) -> np.ndarray:
    r = bf16_round(x).astype(np.float32)   # exact: every bf16 value is a float32
    return (r.view(np.uint32) >> np.uint32(16)).astype(np.uint16)


def bf16_bits_to_f64(b: np.ndarray) -> np.ndarray:
    u = np.asarray(b, dtype=np.uint16).astype(np.uint32) << np.uint32(16)
    return u.view(np.float32).astype(np.float64)


def b_chunk(key: int, nbf: int, naux: int, p0: int, p1: int, dtype: str = "f64") -> np.ndarray:
    """Rows P in [p0, p1) of B, as float64 values (bf16-rounded when dtype == "bf16")."""
    f = b_factor_table(nbf, naux)
    i = np.arange(nbf)
    lo = np.minimum.outer(i, i).astype(np.uint64)
    hi = np.maximum.outer(i, i).astype(np.uint64)
    fac = f[np.abs(np.subtract.outer(i, i))]
    out = np.empty((p1 - p0, nbf, nbf), dtype=np.float64)
    n = np.uint64(nbf)
    for k, P in enumerate(range(p0, p1)):
        idx = (np.uint64(P) * n + lo) * n + hi
        v = fac * ih12(key, idx)
        out[k] = bf16_round(v) if dtype == "bf16" else v
    return out


# ---------------------------------------------------------------- host-side draws
def orthogonal(rng: np.random.Generator, n: int) -> np.ndarray:
    q, _ = np.linalg.qr(rng.standard_normal((n, n)))
    return np.ascontiguousarray(q)


def symmetric_h(rng: np.random.Generator, n: int) -> np.ndarray:
    g = rng.standard_normal((n, n))
    h = np.triu(g, 1)
    h = h + h.T
    h[np.diag_indices(n)] = -rng.uniform(5.0, 20.0, size=n)
    return h


@dataclasses.dataclass
class Instance:
    wl: Workload
    seed: int
    key: int            # counter-stream key of B
    H: np.ndarray
    C: np.ndarray
    gamma: np.ndarray
    B: Optional[np.ndarray] = None     # float64 values (bf16-exact for bf16 workloads)
    ERI: Optional[np.ndarray] = None


def make(wl: Workload, seed: int, stream: int = 0, with_b: bool = True) -> Instance:
    """Draw one instance: H, then C, then gamma from default_rng, then B (P ascending)."""
    rng = np.random.default_rng([seed, stream])
    H = symmetric_h(rng, wl.nbf)
    C = orthogonal(rng, wl.nbf)
    gamma = rng.standard_normal(wl.nact)
    key = stream_key(seed, stream)
    inst = Instance(wl, seed, key, H, C, gamma)
    if with_b or wl.eri4:
        B = b_chunk(key, wl.nbf, wl.naux, 0, wl.naux, wl.b_dtype)
        if wl.eri4:
            n = wl.nbf
            Bm = B.reshape(wl.naux, n * n)
            inst.ERI = np.ascontiguousarray((Bm.T @ Bm).reshape(n, n, n, n))
        if with_b:
            inst.B = B
    return inst


def workload(name: str, with_b: bool = True) -> Instance:
    return make(WORKLOADS[name], seed_of(name), 0, with_b)


def pes_scan(ninst: int = 64, seed: Optional[int] = None, nbf_range=(40, 300), ncwo: int = 3,
             with_b: bool = True) -> list:
    """A batch of independent instances of uneven size (a potential-energy-surface scan).

    nbf ~ integer-uniform in nbf_range (inclusive), naux = 4 nbf, npairs = nbf // 10.
    """
    seed = seed_of("pes64") if seed is None else seed
    rng = np.random.default_rng(seed)
    sizes = rng.integers(nbf_range[0], nbf_range[1] + 1, size=ninst)
    out = []
    for i, n in enumerate(sizes):
        n = int(n)
        wl = Workload(f"pes_{i}", n, 4 * n, n // 10, ncwo, "bf16")
        out.append(make(wl, seed, stream=i + 1, with_b=with_b))
    return out
