"""Python binding of libpnof (include/pnof.h): argument marshalling only.

Every step of the PNOF hot path runs in the HIP library; torch provides device memory and the
stream.  The binding fails loudly when the library is missing: there is no CPU fallback.

Low-level functions carry the C names (``pnof_lagrangian`` ...) and take preallocated torch
tensors; the convenience layer (``Context.lagrangian`` ...) allocates outputs.  Before any call,
tensor sizes, dtypes, devices and contiguity are checked against the problem so that the raw
pointers handed to the library always cover what it will read and write.
"""
from __future__ import annotations

import ctypes
import os
import sys
from typing import Optional

import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
# PNOF_LIBRARY selects another build of the same library (e.g. a debug or variant build)
_LIB_PATH = os.environ.get("PNOF_LIBRARY") or os.path.join(_HERE, "libpnof.so")

PNOF5, PNOF7, PNOF7S = 5, 7, 8
FP64, FP32, BF16, BF16_SPLIT = 0, 1, 2, 3
INTS_ERI4_F64, INTS_DF_F64, INTS_DF_BF16 = 0, 1, 2
CHECK_FINITE = 1
ON_SIGMOID, ON_TRIG = 0, 1
BATCH_GRAPH, BATCH_PERSISTENT = 1, 2

STATUS = {0: "PNOF_OK", 1: "PNOF_E_ARG", 2: "PNOF_E_SHAPE", 3: "PNOF_E_DTYPE", 4: "PNOF_E_NOMEM",
          5: "PNOF_E_DEVICE", 6: "PNOF_E_NONFINITE", 7: "PNOF_E_UNSUPPORTED", 8: "PNOF_E_EIG"}

EXPORTS = ["pnof_abi_version", "pnof_last_error", "pnof_check_problem", "pnof_create", "pnof_destroy",
           "pnof_set_stream", "pnof_workspace_size", "pnof_set_workspace", "pnof_set_pchunk", "pnof_on_map",
           "pnof_on_map_vjp", "pnof_jk", "pnof_energy", "pnof_fock", "pnof_lagrangian", "pnof_orbital_step",
           "pnof_profile_begin", "pnof_profile_end", "pnof_set_tuning", "pnof_get_plan", "pnof_optimize_on",
           "pnof_optimize", "pnof_nofmp2_terms", "pnof_batch_plan",
           "pnof_batch_bind", "pnof_batch_run", "pnof_batch_info", "pnof_batch_destroy", "pnof_batch_set_tiles",
           "pnof_batch_get_tiles", "pnof_batch_times", "pnof_batch_set_stall", "pnof_batch_set_dies",
           "pnof_bind_integrals"]
STAGES = ("X", "b", "Y", "eig")


class PnofError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"{STATUS.get(status, status)}: {msg}")
        self.status = status


class Tuning(ctypes.Structure):
    _fields_ = [(n, ctypes.c_int32) for n in ("pchunk", "nsplit_b", "nsplit_y", "x_variant", "y_variant")]

    def as_dict(self):
        return {n: getattr(self, n) for n, _ in self._fields_}


class OnOpts(ctypes.Structure):
    _fields_ = [("maxiter", ctypes.c_int32), ("memory", ctypes.c_int32), ("gtol", ctypes.c_double)]


class OptOpts(ctypes.Structure):
    _fields_ = [("on_kind", ctypes.c_int32), ("maxit", ctypes.c_int32), ("ndiis", ctypes.c_int32),
                ("fix_n", ctypes.c_int32), ("eps_n", ctypes.c_double), ("eps_phi", ctypes.c_double),
                ("eps", ctypes.c_double), ("delta", ctypes.c_double), ("zeta", ctypes.c_double), ("on", OnOpts)]


class OptResult(ctypes.Structure):
    _fields_ = [("E", ctypes.c_double), ("max_asym", ctypes.c_double), ("d_n", ctypes.c_double),
                ("d_phi", ctypes.c_double), ("d_E", ctypes.c_double), ("iterations", ctypes.c_int32),
                ("converged", ctypes.c_int32)]

    def as_dict(self):
        return {n: getattr(self, n) for n, _ in self._fields_}


class BatchIO(ctypes.Structure):
    _fields_ = [(n, ctypes.c_void_p) for n in ("C", "n", "H", "ints", "lambda_", "E", "dEdC", "dEdn", "max_asym",
                                                "gamma", "dEdgamma")] + [("on_kind", ctypes.c_int32)]


class Problem(ctypes.Structure):
    _fields_ = [(n, ctypes.c_int32) for n in
                ("nbf", "naux", "npairs", "ncwo", "functional", "precision", "ints", "flags", "nsingle")]

    @property
    def nact(self) -> int:
        return self.npairs * (self.ncwo + 1) + self.nsingle


_lib = None


def library_path() -> str:
    return _LIB_PATH


def lib():
    """Load libpnof.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            raise ImportError(f"{_LIB_PATH} is missing: run `python -m paper_2004_06142_amd.build`")
        L = ctypes.CDLL(_LIB_PATH)
        P, I, D, S = ctypes.c_void_p, ctypes.c_int32, ctypes.c_double, ctypes.c_int
        PP = ctypes.POINTER(Problem)
        sig = {
            "pnof_abi_version": ([], S),
            "pnof_last_error": ([P], ctypes.c_char_p),
            "pnof_check_problem": ([PP], S),
            "pnof_create": ([ctypes.POINTER(ctypes.c_void_p), S, P], S),
            "pnof_destroy": ([P], None),
            "pnof_set_stream": ([P, P], S),
            "pnof_workspace_size": ([P, PP, ctypes.POINTER(ctypes.c_size_t)], S),
            "pnof_set_workspace": ([P, P, ctypes.c_size_t], S),
            "pnof_set_pchunk": ([P, I], S),
            "pnof_bind_integrals": ([P, PP, P], S),
            "pnof_on_map": ([P, I, I, I, I, P, P, P], S),
            "pnof_on_map_vjp": ([P, I, I, I, I, P, P, P], S),
            "pnof_jk": ([P, PP, P, P, P, P, P, P, P, I], S),
            "pnof_energy": ([P, PP, P, P, P, P, P], S),
            "pnof_fock": ([P, PP, P, P, P, P, P, P, P, I], S),
            "pnof_lagrangian": ([P, PP, P, P, P, P, P, P, P, P, P, P, P], S),
            "pnof_lagrangian_noalloc": ([P, PP, P, P, P, P, P, P, P, P, P, P, P], S),
            "pnof_orbital_step": ([P, I, P, P, P, D, P, P, P], S),
            "pnof_set_tuning": ([P, ctypes.POINTER(Tuning)], S),
            "pnof_get_plan": ([P, PP, ctypes.POINTER(Tuning)], S),
            "pnof_profile_begin": ([P], S),
            "pnof_profile_end": ([P, ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_int64)], S),
            "pnof_optimize_on": ([P, PP, I, P, P, P, P, P, ctypes.POINTER(OnOpts), ctypes.POINTER(ctypes.c_double),
                                  ctypes.POINTER(ctypes.c_int32)], S),
            "pnof_optimize": ([P, PP, P, P, P, P, P, ctypes.POINTER(OptOpts), ctypes.POINTER(OptResult)], S),
            "pnof_nofmp2_terms": ([P, PP, P, P, P, P, P, P], S),
            "pnof_batch_plan": ([P, I, PP, ctypes.POINTER(ctypes.c_void_p)], S),
            "pnof_batch_bind": ([P, ctypes.POINTER(BatchIO)], S),
            "pnof_batch_run": ([P, I], S),
            "pnof_batch_info": ([P, ctypes.POINTER(ctypes.c_size_t), ctypes.POINTER(ctypes.c_int32)], S),
            "pnof_batch_destroy": ([P], None),
            "pnof_batch_set_tiles": ([P, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32], S),
            "pnof_batch_get_tiles": ([P, ctypes.POINTER(ctypes.c_int32)], S),
            "pnof_batch_times": ([P, ctypes.POINTER(ctypes.c_double)], S),
            "pnof_batch_set_stall": ([P, ctypes.c_double], S),
            "pnof_batch_set_dies": ([P, I], S),
        }
        for name, (args, res) in sig.items():
            f = getattr(L, name)
            f.argtypes = args
            f.restype = res
        _lib = L
    return _lib


def problem(nbf, naux, npairs, ncwo, functional=PNOF7, precision=FP64, ints=INTS_DF_F64, flags=0,
            nsingle=0) -> Problem:
    return Problem(nbf, naux, npairs, ncwo, functional, precision, ints, flags, nsingle)


# ----------------------------------------------------------------------------- marshalling
def _ptr(t: Optional[torch.Tensor]):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


def _check(t: Optional[torch.Tensor], numel: int, dtype, device, name: str, optional=False):
    if t is None:
        if optional:
            return
        raise ValueError(f"{name} is required")
    if t.dtype != dtype:
        raise TypeError(f"{name}: expected {dtype}, got {t.dtype}")
    if t.device != device:
        raise ValueError(f"{name}: expected device {device}, got {t.device}")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    if t.numel() != numel:
        raise ValueError(f"{name}: expected {numel} elements, got {t.numel()}")


def _ints_check(prob: Problem, ints: torch.Tensor, device):
    if prob.ints == INTS_ERI4_F64:
        _check(ints, prob.nbf ** 4, torch.float64, device, "ERI")
    elif prob.ints == INTS_DF_F64:
        _check(ints, prob.naux * prob.nbf ** 2, torch.float64, device, "B")
    else:
        _check(ints, prob.naux * prob.nbf ** 2, torch.bfloat16, device, "B")


def _raise(ctx, st):
    if st != 0:
        msg = lib().pnof_last_error(ctx.handle if ctx is not None else None)
        raise PnofError(st, msg.decode() if msg else "")


class Context:
    """A libpnof context on one device, issuing work on torch's current stream of that device."""

    def __init__(self, device: int = 0, stream: Optional[torch.cuda.Stream] = None):
        L = lib()
        self.device = torch.device("cuda", device)
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        h = ctypes.c_void_p()
        st = L.pnof_create(ctypes.byref(h), device, ctypes.c_void_p(self.stream.cuda_stream))
        if st != 0:
            raise PnofError(st, L.pnof_last_error(None).decode())
        self.handle = h
        self._ws = None

    def close(self):
        if getattr(self, "handle", None):
            lib().pnof_destroy(self.handle)
            self.handle = None

    def __del__(self, _finalizing=sys.is_finalizing):
        # at interpreter shutdown the HIP runtime may already be tearing down: the process's end
        # releases the device resources instead
        if _finalizing():
            return
        try:
            self.close()
        except Exception:
            pass

    def profile_begin(self):
        _raise(self, lib().pnof_profile_begin(self.handle))

    def profile_end(self):
        """Per-stage (X, b, Y, eig) summed event milliseconds and launch counts since profile_begin."""
        ms = (ctypes.c_double * 4)()
        cnt = (ctypes.c_int64 * 4)()
        _raise(self, lib().pnof_profile_end(self.handle, ms, cnt))
        return {k: (ms[i], cnt[i]) for i, k in enumerate(STAGES)}

    def set_tuning(self, tuning=None, **kw):
        """Set launch parameters (a Tuning, a dict, or keywords); None resets to automatic."""
        if tuning is None and not kw:
            _raise(self, lib().pnof_set_tuning(self.handle, None))
            return
        t = tuning if isinstance(tuning, Tuning) else Tuning(**{**(tuning or {}), **kw})
        _raise(self, lib().pnof_set_tuning(self.handle, ctypes.byref(t)))

    def plan(self, prob) -> dict:
        t = Tuning()
        _raise(self, lib().pnof_get_plan(self.handle, ctypes.byref(prob), ctypes.byref(t)))
        return t.as_dict()

    def set_pchunk(self, pc: int):
        _raise(self, lib().pnof_set_pchunk(self.handle, pc))

    def bind_integrals(self, prob: Optional[Problem] = None, ints: Optional[torch.Tensor] = None):
        """Keep the split mode's row bounds of `ints` for later calls on the same integrals
        (pnof_bind_integrals); no arguments unbind.  The bound tensor must not change while bound."""
        if prob is None or ints is None:
            _raise(self, lib().pnof_bind_integrals(self.handle, None, None))
            return
        _ints_check(prob, ints, self.device)
        _raise(self, lib().pnof_bind_integrals(self.handle, ctypes.byref(prob), _ptr(ints)))

    def reserve(self, prob: Problem):
        """Allocate the workspace for `prob` as a torch tensor and lend it to the library."""
        n = ctypes.c_size_t()
        _raise(self, lib().pnof_workspace_size(self.handle, ctypes.byref(prob), ctypes.byref(n)))
        self._ws = torch.empty(n.value + 256, dtype=torch.uint8, device=self.device)
        base = self._ws.data_ptr()
        off = (-base) % 256
        _raise(self, lib().pnof_set_workspace(self.handle, ctypes.c_void_p(base + off), n.value))
        return n.value

    # ------------------------------------------------------------------ convenience layer
    def _f64(self, *shape):
        return torch.empty(*shape, dtype=torch.float64, device=self.device)

    def on_map(self, gamma, npairs, ncwo, kind=ON_SIGMOID, jacobian=False, nsingle=0):
        nact = npairs * (ncwo + 1) + nsingle
        ngam = nact if kind == ON_SIGMOID else npairs * ncwo
        n = self._f64(nact)
        jac = self._f64(nact, ngam) if jacobian else None
        pnof_on_map(self, kind, npairs, ncwo, gamma, n, jac, nsingle)
        return (n, jac) if jacobian else n

    def on_map_vjp(self, gamma, dEdn, npairs, ncwo, kind=ON_SIGMOID, nsingle=0):
        out = self._f64(gamma.numel())
        pnof_on_map_vjp(self, kind, npairs, ncwo, gamma, dEdn, out, nsingle)
        return out

    def jk(self, prob, C, ints, q_idx=None):
        J, K = self._f64(prob.nact, prob.nact), self._f64(prob.nact, prob.nact)
        Jq = Kq = None
        if q_idx is not None:
            Jq, Kq = self._f64(len(q_idx), prob.nbf, prob.nbf), self._f64(len(q_idx), prob.nbf, prob.nbf)
        pnof_jk(self, prob, C, ints, J, K, Jq, Kq, q_idx)
        return (J, K) if q_idx is None else (J, K, Jq, Kq)

    def energy(self, prob, C, n, H, ints):
        E = self._f64(1)
        pnof_energy(self, prob, C, n, H, ints, E)
        return E

    def fock(self, prob, C, n, H, ints, q_idx=None):
        Y = self._f64(prob.nbf, prob.nact)
        Fq = self._f64(len(q_idx), prob.nbf, prob.nbf) if q_idx is not None else None
        pnof_fock(self, prob, C, n, H, ints, Y, Fq, q_idx)
        return Y if q_idx is None else (Y, Fq)

    def lagrangian(self, prob, C, n, H, ints, grads=True, jk=False):
        nbf, nact = prob.nbf, prob.nact
        out = {"lam": self._f64(nbf, nbf), "E": self._f64(1), "max_asym": self._f64(1)}
        if grads:
            out["dEdC"] = self._f64(nbf, nbf)
            out["dEdn"] = self._f64(nact)
        if jk:
            out["J"] = self._f64(nact, nact)
            out["K"] = self._f64(nact, nact)
        pnof_lagrangian(self, prob, C, n, H, ints, out["lam"], out["E"], out.get("dEdC"), out.get("dEdn"),
                        out["max_asym"], out.get("J"), out.get("K"))
        return out

    def nofmp2_terms(self, prob, C, n, H, ints):
        """(E_hf, E_sta) device scalars of Eqs. HFL and Esta."""
        d = self.device
        for tt, name in ((C, "C"), (H, "H")):
            _check(tt, prob.nbf ** 2, torch.float64, d, name)
        _check(n, prob.nact, torch.float64, d, "n")
        _ints_check(prob, ints, d)
        e_hf, e_sta = self._f64(1), self._f64(1)
        _raise(self, lib().pnof_nofmp2_terms(self.handle, ctypes.byref(prob), _ptr(C), _ptr(n), _ptr(H), _ptr(ints),
                                             _ptr(e_hf), _ptr(e_sta)))
        return e_hf, e_sta

    def optimize_on(self, prob, C, H, J, K, gamma, kind=ON_SIGMOID, maxiter=0, memory=0, gtol=0.0):
        """Occupation optimisation at fixed orbitals; returns (gamma, E, iterations) (gamma copied)."""
        d = self.device
        nbf, nact = prob.nbf, prob.nact
        ngam = nact if kind == ON_SIGMOID else prob.npairs * prob.ncwo
        for t, name in ((C, "C"), (H, "H")):
            _check(t, nbf * nbf, torch.float64, d, name)
        for t, name in ((J, "J"), (K, "K")):
            _check(t, nact * nact, torch.float64, d, name)
        _check(gamma, ngam, torch.float64, d, "gamma")
        g = gamma.clone()
        E, it = ctypes.c_double(), ctypes.c_int32()
        opts = OnOpts(maxiter, memory, gtol)
        _raise(self, lib().pnof_optimize_on(self.handle, ctypes.byref(prob), kind, _ptr(C), _ptr(H), _ptr(J), _ptr(K),
                                            _ptr(g), ctypes.byref(opts), ctypes.byref(E), ctypes.byref(it)))
        return g, E.value, it.value

    def optimize(self, prob, H, ints, C, gamma=None, n=None, on_kind=ON_SIGMOID, maxit=200, ndiis=0, fix_n=False,
                 eps_n=0.0, eps_phi=0.0, eps=0.0, delta=1e-4, zeta=0.0, on_maxiter=0, on_gtol=0.0):
        """Orbital + occupation optimisation (Section 3.4).  Returns dict with C, gamma, n and the
        result fields (E, max_asym, d_n, d_phi, d_E, iterations, converged); inputs are not modified."""
        d = self.device
        nbf, nact = prob.nbf, prob.nact
        _check(H, nbf * nbf, torch.float64, d, "H")
        _check(C, nbf * nbf, torch.float64, d, "C")
        _ints_check(prob, ints, d)
        Cw = C.clone()
        nw = n.clone() if n is not None else self._f64(nact)
        _check(nw, nact, torch.float64, d, "n")
        gw = None
        if not fix_n:
            ngam = nact if on_kind == ON_SIGMOID else prob.npairs * prob.ncwo
            _check(gamma, ngam, torch.float64, d, "gamma")
            gw = gamma.clone()
        elif n is None:
            raise ValueError("fix_n needs n")
        opts = OptOpts(on_kind, maxit, ndiis, 1 if fix_n else 0, eps_n, eps_phi, eps, delta, zeta,
                       OnOpts(on_maxiter, 0, on_gtol))
        res = OptResult()
        _raise(self, lib().pnof_optimize(self.handle, ctypes.byref(prob), _ptr(H), _ptr(ints), _ptr(Cw), _ptr(gw),
                                         _ptr(nw), ctypes.byref(opts), ctypes.byref(res)))
        return {"C": Cw, "gamma": gw, "n": nw, **res.as_dict()}

    def orbital_step(self, lam, C, diag_prev=None, zeta=0.0, want_s=False):
        nbf = C.shape[0]
        Cn, eps = self._f64(nbf, nbf), self._f64(nbf)
        S = self._f64(nbf, nbf) if want_s else None
        pnof_orbital_step(self, nbf, lam, C, diag_prev, zeta, Cn, eps, S)
        return (Cn, eps, S) if want_s else (Cn, eps)


# ----------------------------------------------------------------------------- C-named calls
def pnof_check_problem(prob: Problem) -> int:
    return lib().pnof_check_problem(ctypes.byref(prob))


def pnof_on_map(ctx, kind, npairs, ncwo, gamma, n, dn_dgamma=None, nsingle=0):
    nact = npairs * (ncwo + 1) + nsingle
    ngam = nact if kind == ON_SIGMOID else npairs * ncwo
    _check(gamma, ngam, torch.float64, ctx.device, "gamma")
    _check(n, nact, torch.float64, ctx.device, "n")
    _check(dn_dgamma, nact * ngam, torch.float64, ctx.device, "dn_dgamma", optional=True)
    _raise(ctx, lib().pnof_on_map(ctx.handle, kind, npairs, ncwo, nsingle, _ptr(gamma), _ptr(n), _ptr(dn_dgamma)))


def pnof_on_map_vjp(ctx, kind, npairs, ncwo, gamma, dEdn, dEdgamma, nsingle=0):
    nact = npairs * (ncwo + 1) + nsingle
    ngam = nact if kind == ON_SIGMOID else npairs * ncwo
    _check(gamma, ngam, torch.float64, ctx.device, "gamma")
    _check(dEdn, nact, torch.float64, ctx.device, "dEdn")
    _check(dEdgamma, ngam, torch.float64, ctx.device, "dEdgamma")
    _raise(ctx, lib().pnof_on_map_vjp(ctx.handle, kind, npairs, ncwo, nsingle, _ptr(gamma), _ptr(dEdn),
                                      _ptr(dEdgamma)))


def _q(ctx, prob, q_idx):
    if q_idx is None:
        return None, 0
    q = torch.as_tensor(q_idx, dtype=torch.int32).to(ctx.device).contiguous()
    if q.numel() == 0 or int(q.min()) < 0 or int(q.max()) >= prob.nact:
        raise ValueError("q_idx entries must lie in [0, nact)")
    return q, q.numel()


def pnof_jk(ctx, prob, C, ints, J, K, Jq_ao=None, Kq_ao=None, q_idx=None):
    d = ctx.device
    _check(C, prob.nbf ** 2, torch.float64, d, "C")
    _ints_check(prob, ints, d)
    _check(J, prob.nact ** 2, torch.float64, d, "J")
    _check(K, prob.nact ** 2, torch.float64, d, "K")
    q, nq = _q(ctx, prob, q_idx)
    _check(Jq_ao, nq * prob.nbf ** 2, torch.float64, d, "Jq_ao", optional=True)
    _check(Kq_ao, nq * prob.nbf ** 2, torch.float64, d, "Kq_ao", optional=True)
    _raise(ctx, lib().pnof_jk(ctx.handle, ctypes.byref(prob), _ptr(C), _ptr(ints), _ptr(J), _ptr(K), _ptr(Jq_ao),
                              _ptr(Kq_ao), _ptr(q), nq))


def _common(ctx, prob, C, n, H, ints):
    d = ctx.device
    _check(C, prob.nbf ** 2, torch.float64, d, "C")
    if n is None or n.dtype != torch.float64 or n.device != d or not n.is_contiguous() or n.numel() < prob.nact:
        raise ValueError("n: float64 contiguous device tensor with at least nact entries required")
    _check(H, prob.nbf ** 2, torch.float64, d, "H")
    _ints_check(prob, ints, d)


def pnof_energy(ctx, prob, C, n, H, ints, E):
    _common(ctx, prob, C, n, H, ints)
    _check(E, 1, torch.float64, ctx.device, "E")
    _raise(ctx, lib().pnof_energy(ctx.handle, ctypes.byref(prob), _ptr(C), _ptr(n), _ptr(H), _ptr(ints), _ptr(E)))


def pnof_fock(ctx, prob, C, n, H, ints, Y, Fq_ao=None, q_idx=None):
    _common(ctx, prob, C, n, H, ints)
    _check(Y, prob.nbf * prob.nact, torch.float64, ctx.device, "Y")
    q, nq = _q(ctx, prob, q_idx)
    _check(Fq_ao, nq * prob.nbf ** 2, torch.float64, ctx.device, "Fq_ao", optional=True)
    _raise(ctx, lib().pnof_fock(ctx.handle, ctypes.byref(prob), _ptr(C), _ptr(n), _ptr(H), _ptr(ints), _ptr(Y),
                                _ptr(Fq_ao), _ptr(q), nq))


def pnof_lagrangian(ctx, prob, C, n, H, ints, lam, E, dEdC=None, dEdn=None, max_asym=None, J=None, K=None):
    _common(ctx, prob, C, n, H, ints)
    d = ctx.device
    _check(lam, prob.nbf ** 2, torch.float64, d, "lambda")
    _check(E, 1, torch.float64, d, "E")
    _check(dEdC, prob.nbf ** 2, torch.float64, d, "dEdC", optional=True)
    _check(dEdn, prob.nact, torch.float64, d, "dEdn", optional=True)
    _check(max_asym, 1, torch.float64, d, "max_asym", optional=True)
    _check(J, prob.nact ** 2, torch.float64, d, "J", optional=True)
    _check(K, prob.nact ** 2, torch.float64, d, "K", optional=True)
    _raise(ctx, lib().pnof_lagrangian(ctx.handle, ctypes.byref(prob), _ptr(C), _ptr(n), _ptr(H), _ptr(ints),
                                      _ptr(lam), _ptr(E), _ptr(dEdC), _ptr(dEdn), _ptr(max_asym), _ptr(J), _ptr(K)))


def pnof_orbital_step(ctx, nbf, lam, C, diag_prev, zeta, C_new, eps, S_out=None):
    d = ctx.device
    for t, name in ((lam, "lambda"), (C, "C"), (C_new, "C_new")):
        _check(t, nbf * nbf, torch.float64, d, name)
    _check(eps, nbf, torch.float64, d, "eps")
    _check(diag_prev, nbf, torch.float64, d, "diag_prev", optional=True)
    _check(S_out, nbf * nbf, torch.float64, d, "S_out", optional=True)
    _raise(ctx, lib().pnof_orbital_step(ctx.handle, nbf, _ptr(lam), _ptr(C), _ptr(diag_prev), float(zeta),
                                        _ptr(C_new), _ptr(eps), _ptr(S_out)))


# ----------------------------------------------------------------------------- autograd
class PNOFEnergy(torch.autograd.Function):
    """E(C, gamma) with the device adjoint: dE/dC = 4 F^q c_q, dE/dgamma = (dn/dgamma)^T dE/dn.

    Both gradients come out of the same forward pass (Lagrangian kernels and the ON-map adjoint
    kernel); backward only scales them by the incoming gradient.
    """

    @staticmethod
    def forward(fctx, C, gamma, H, ints, prob, ctx, kind=ON_SIGMOID):
        n = ctx.on_map(gamma, prob.npairs, prob.ncwo, kind, nsingle=prob.nsingle)
        out = ctx.lagrangian(prob, C, n, H, ints, grads=True)
        dEdg = ctx.on_map_vjp(gamma, out["dEdn"], prob.npairs, prob.ncwo, kind, nsingle=prob.nsingle)
        fctx.save_for_backward(out["dEdC"], dEdg)
        return out["E"].reshape(())

    @staticmethod
    def backward(fctx, gE):
        dEdC, dEdg = fctx.saved_tensors
        return gE * dEdC, gE * dEdg, None, None, None, None, None


def energy_and_grad(ctx, prob, C, gamma, H, ints, kind=ON_SIGMOID):
    """One energy + gradient evaluation (forward of PNOFEnergy), returning all device outputs."""
    n = ctx.on_map(gamma, prob.npairs, prob.ncwo, kind, nsingle=prob.nsingle)
    out = ctx.lagrangian(prob, C, n, H, ints, grads=True)
    out["dEdgamma"] = ctx.on_map_vjp(gamma, out["dEdn"], prob.npairs, prob.ncwo, kind, nsingle=prob.nsingle)
    out["n"] = n
    return out


# ----------------------------------------------------------------------------- batches
class Batch:
    """A batch of independent problems, run as one fixed sequence of grouped launches or as one
    persistent launch.

    ``problems``: list of Problem (DF_BF16, one precision).  ``bind(inputs)`` takes, per instance, a
    dict with device tensors C, n, H, B and optionally gamma (with ``on_kind``, for dE/dgamma), and
    allocates the outputs (dEdC / dEdn / max_asym / dEdgamma with ``grads=True``).  ``run(graph,
    persistent)`` enqueues one step of every instance (with ``graph``, captured into a HIP graph on
    the first call) and returns the output dicts; after a persistent run ``times()`` gives each
    instance's completion time in microseconds after the run's start.
    """

    def __init__(self, ctx: Context, problems):
        self.ctx = ctx
        self.problems = list(problems)
        arr = (Problem * len(self.problems))(*self.problems)
        h = ctypes.c_void_p()
        _raise(ctx, lib().pnof_batch_plan(ctx.handle, len(self.problems), arr, ctypes.byref(h)))
        self.handle = h
        self.inputs = None
        self.outputs = None

    def info(self):
        nb, nl = ctypes.c_size_t(), ctypes.c_int32()
        _raise(self.ctx, lib().pnof_batch_info(self.handle, ctypes.byref(nb), ctypes.byref(nl)))
        return {"bytes": nb.value, "launches": nl.value}

    def set_tiles(self, x: int = 0, b: int = 0, y: int = 0):
        """Tile widths (64 or 128; 0 = automatic) along the active orbitals of the grouped X, b, Y."""
        _raise(self.ctx, lib().pnof_batch_set_tiles(self.handle, x, b, y))

    def tiles(self) -> tuple:
        out = (ctypes.c_int32 * 3)()
        _raise(self.ctx, lib().pnof_batch_get_tiles(self.handle, out))
        return tuple(out)

    def bind(self, inputs, grads: bool = True):
        if len(inputs) != len(self.problems):
            raise ValueError("one input dict per instance is required")
        d = self.ctx.device
        ios = (BatchIO * len(inputs))()
        outs = []
        for i, (prob, x) in enumerate(zip(self.problems, inputs)):
            nbf = prob.nbf
            _check(x["C"], nbf * nbf, torch.float64, d, f"C[{i}]")
            _check(x["H"], nbf * nbf, torch.float64, d, f"H[{i}]")
            if x["n"].numel() not in (prob.nact, nbf):
                raise ValueError(f"n[{i}]: expected nact or nbf entries")
            _check(x["n"], x["n"].numel(), torch.float64, d, f"n[{i}]")
            _ints_check(prob, x["B"], d)
            o = {"E": torch.zeros(1, dtype=torch.float64, device=d),
                 "lam": torch.zeros(nbf, nbf, dtype=torch.float64, device=d)}
            gam = x.get("gamma")
            kind = int(x.get("on_kind", ON_SIGMOID))
            if gam is not None and kind in (ON_SIGMOID, ON_TRIG):   # the library rejects other kinds
                ngam = prob.nact if kind == ON_SIGMOID else prob.npairs * prob.ncwo
                _check(gam, ngam, torch.float64, d, f"gamma[{i}]")
            if grads:
                o["dEdC"] = torch.zeros(nbf, nbf, dtype=torch.float64, device=d)
                o["dEdn"] = torch.zeros(prob.nact, dtype=torch.float64, device=d)
                o["max_asym"] = torch.zeros(1, dtype=torch.float64, device=d)
                if gam is not None:
                    o["dEdgamma"] = torch.zeros(gam.numel(), dtype=torch.float64, device=d)
            io = ios[i]
            io.C, io.n, io.H, io.ints = (x["C"].data_ptr(), x["n"].data_ptr(), x["H"].data_ptr(), x["B"].data_ptr())
            io.lambda_, io.E = o["lam"].data_ptr(), o["E"].data_ptr()
            io.dEdC = o["dEdC"].data_ptr() if grads else None
            io.dEdn = o["dEdn"].data_ptr() if grads else None
            io.max_asym = o["max_asym"].data_ptr() if grads else None
            io.gamma = gam.data_ptr() if gam is not None else None
            io.dEdgamma = o["dEdgamma"].data_ptr() if "dEdgamma" in o else None
            io.on_kind = kind
            outs.append(o)
        _raise(self.ctx, lib().pnof_batch_bind(self.handle, ios))
        self.inputs, self.outputs = list(inputs), outs   # keep the bound tensors alive
        return outs

    def run(self, graph: bool = True, persistent: bool = False):
        flags = (BATCH_GRAPH if graph else 0) | (BATCH_PERSISTENT if persistent else 0)
        _raise(self.ctx, lib().pnof_batch_run(self.handle, flags))
        return self.outputs

    def times(self):
        """Completion time of each instance in the last persistent run (microseconds after its
        start); synchronises the context stream."""
        out = (ctypes.c_double * len(self.problems))()
        _raise(self.ctx, lib().pnof_batch_times(self.handle, out))
        return list(out)

    def set_dies(self, dies: int = 0):
        """Die groups of the persistent form (0: the device's XCC count)."""
        _raise(self.ctx, lib().pnof_batch_set_dies(self.handle, int(dies)))

    def set_stall(self, microseconds: float = 0.0):
        """Time with no progress anywhere before a persistent run's blocks give up (0: one second)."""
        _raise(self.ctx, lib().pnof_batch_set_stall(self.handle, float(microseconds)))

    def close(self):
        if getattr(self, "handle", None):
            lib().pnof_batch_destroy(self.handle)
            self.handle = None

    def __del__(self, _finalizing=sys.is_finalizing):
        # at interpreter shutdown the HIP runtime may already be tearing down: the process's end
        # releases the device resources instead
        if _finalizing():
            return
        try:
            self.close()
        except Exception:
            pass
