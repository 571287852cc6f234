"""Thin ctypes binding of the C ABI in include/ls.h.

Argument marshalling only: every step of the solver runs in the HIP library
``libls.so`` built from csrc/.  Torch is used for device memory and streams:
fields are passed as contiguous CUDA (HIP) tensors and the current torch
stream is handed to the library.  There is no fallback: if the library is
missing, ``load()`` raises.
"""
from __future__ import annotations

import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libls.so")

LS_C128, LS_C64, LS_MIXED = 0, 1, 2
PREC = {"c128": LS_C128, "c64": LS_C64, "mixed": LS_MIXED}


class LSError(RuntimeError):
    def __init__(self, code: int, what: str):
        self.code = code
        msg = _lib.ls_status_string(code).decode() if _lib is not None else str(code)
        super().__init__(f"{what}: {msg} ({code})")


class PlanDesc(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int), ("k", ctypes.c_double), ("max_rhs", ctypes.c_int),
                ("host_mem_cap", ctypes.c_size_t), ("tune_cache", ctypes.c_char_p)]


_lib = None

# (name, restype, argtypes) of every exported entry point
_VP, _I, _D = ctypes.c_void_p, ctypes.c_int, ctypes.c_double
SIGNATURES = [
    ("ls_status_string", ctypes.c_char_p, [_I]),
    ("ls_plan_create", _I, [ctypes.POINTER(PlanDesc), _VP, _VP, ctypes.POINTER(_VP)]),
    ("ls_apply", _I, [_VP, _VP, _VP, _I, _I, _VP]),
    ("ls_apply_timed", _I, [_VP, _VP, _VP, _I, _I, _VP, ctypes.POINTER(ctypes.c_double)]),
    ("ls_rhs_from_incident", _I, [_VP, _VP, _VP, _I, _VP]),
    ("ls_plan_fft_size", _I, [_VP]),
    ("ls_plan_destroy", None, [_VP]),
]


def load(path: str = LIB_PATH):
    """Load libls.so (raises OSError when it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise OSError(f"HIP library not built: {path} (run __graft_entry__.build())")
    lib = ctypes.CDLL(path)
    for name, res, args in SIGNATURES:
        f = getattr(lib, name)
        f.restype = res
        f.argtypes = args
    _lib = lib
    return lib


def _check(code: int, what: str):
    if code != 0:
        raise LSError(code, what)


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr())


def _stream():
    import torch
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def _field(t, dtype, n, name):
    import torch
    if not t.is_cuda or t.dtype != dtype or not t.is_contiguous():
        raise ValueError(f"{name}: need a contiguous CUDA tensor of {dtype}")
    if t.dim() != 5 or tuple(t.shape[1:]) != (3, n, n, n):
        raise ValueError(f"{name}: shape must be (nrhs, 3, {n}, {n}, {n}), got {tuple(t.shape)}")
    return t


class Plan:
    """A solver plan: contrast, Khat and workspaces on the GPU."""

    def __init__(self, n: int, k: float, m, max_rhs: int = 1, host_mem_cap: int = 0,
                 tune_cache: str | None = None):
        import torch
        lib = load()
        if m.dtype != torch.complex128 or not m.is_cuda or tuple(m.shape) != (n, n, n):
            raise ValueError("m must be a (n, n, n) complex128 CUDA tensor")
        m = m.contiguous()
        self.n, self.k, self.max_rhs = n, float(k), max_rhs
        desc = PlanDesc(n, float(k), max_rhs, host_mem_cap,
                        tune_cache.encode() if tune_cache else None)
        h = ctypes.c_void_p()
        _check(lib.ls_plan_create(ctypes.byref(desc), _ptr(m), _stream(), ctypes.byref(h)),
               "ls_plan_create")
        self._h = h
        self.P = lib.ls_plan_fft_size(h)

    def close(self):
        if getattr(self, "_h", None):
            _lib.ls_plan_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def apply(self, x, y=None, prec: str = "c128"):
        """y = x + K * (m x) (Eq. (5)); x complex128 (c128, mixed) or complex64 (c64)."""
        import torch
        dt = torch.complex64 if prec == "c64" else torch.complex128
        _field(x, dt, self.n, "x")
        if y is None:
            y = torch.empty_like(x)
        _field(y, dt, self.n, "y")
        _check(_lib.ls_apply(self._h, _ptr(x), _ptr(y), x.shape[0], PREC[prec], _stream()),
               "ls_apply")
        return y

    def apply_timed(self, x, y, prec: str = "c128"):
        """ls_apply with per-pass GPU milliseconds (list of 5)."""
        import torch
        dt = torch.complex64 if prec == "c64" else torch.complex128
        _field(x, dt, self.n, "x")
        _field(y, dt, self.n, "y")
        ms = (ctypes.c_double * 5)()
        _check(_lib.ls_apply_timed(self._h, _ptr(x), _ptr(y), x.shape[0], PREC[prec], _stream(), ms),
               "ls_apply_timed")
        return list(ms)

    def rhs_from_incident(self, Ei, g=None):
        """g = -K * (m E^i) (right-hand side of Eq. (4)), complex128."""
        import torch
        _field(Ei, torch.complex128, self.n, "Ei")
        if g is None:
            g = torch.empty_like(Ei)
        _check(_lib.ls_rhs_from_incident(self._h, _ptr(Ei), _ptr(g), Ei.shape[0], _stream()),
               "ls_rhs_from_incident")
        return g
