"""Device-side generation of B (same values as ``synth.b_chunk``, bit for bit)."""
from __future__ import annotations

import ctypes
import os

import numpy as np
import torch

from . import b_factor_table

_LIB = os.path.join(os.path.dirname(os.path.abspath(__file__)), "_synthdev.so")
_lib = None


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            raise ImportError(f"{_LIB} is missing: run `python -m synth.build`")
        L = ctypes.CDLL(_LIB)
        L.synth_fill_b.argtypes = [ctypes.c_void_p, ctypes.c_int, ctypes.c_void_p, ctypes.c_uint64,
                                   ctypes.c_int64, ctypes.c_int64, ctypes.c_int64, ctypes.c_void_p]
        L.synth_fill_b.restype = ctypes.c_int
        _lib = L
    return _lib


def fill_b(out: torch.Tensor, key: int, nbf: int, naux: int, p0: int = 0, stream=None) -> torch.Tensor:
    """Fill ``out`` (shape (nP, nbf, nbf), float64 or bfloat16, on a GPU) with rows p0..p0+nP of B."""
    if out.dim() != 3 or out.shape[1] != nbf or out.shape[2] != nbf or not out.is_contiguous():
        raise ValueError("out must be a contiguous (nP, nbf, nbf) tensor")
    if out.dtype not in (torch.float64, torch.bfloat16):
        raise TypeError("out must be float64 or bfloat16")
    if p0 < 0 or p0 + out.shape[0] > naux:
        raise ValueError("rows outside [0, naux)")
    fac = torch.from_numpy(b_factor_table(nbf, naux)).to(out.device)
    s = stream if stream is not None else torch.cuda.current_stream(out.device)
    rc = _load().synth_fill_b(ctypes.c_void_p(out.data_ptr()), int(out.dtype == torch.bfloat16),
                              ctypes.c_void_p(fac.data_ptr()), ctypes.c_uint64(key), nbf, p0, out.shape[0],
                              ctypes.c_void_p(s.cuda_stream))
    if rc != 0:
        raise RuntimeError(f"synth_fill_b failed with HIP error {rc}")
    s.synchronize()   # keeps `fac` alive until the kernel has run
    return out


def make_b(key: int, nbf: int, naux: int, dtype=torch.bfloat16, device="cuda") -> torch.Tensor:
    out = torch.empty((naux, nbf, nbf), dtype=dtype, device=device)
    return fill_b(out, key, nbf, naux)


def to_numpy_f64(t: torch.Tensor) -> np.ndarray:
    return t.to(torch.float64).cpu().numpy()
