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
    ("ls_stencil_fit", _I, [_VP, _I, _VP]),
    ("ls_get_class_stencils", _I, [_VP, _VP, _VP, _VP, _VP]),
    ("ls_get_point_stencils", _I, [_VP, _VP, _VP]),
    ("ls_get_rows", _I, [_VP, _VP]),
    ("ls_factor", _I, [_VP, ctypes.POINTER(ctypes.c_double)]),
    ("ls_factor_prec", _I, [_VP, _I, ctypes.POINTER(ctypes.c_double)]),
    ("ls_factor_gpu", _I, [_VP, _I, _VP, ctypes.POINTER(ctypes.c_double)]),
    ("ls_precond_apply", _I, [_VP, _VP, _VP, _I, _VP]),
    ("ls_gmres_solve", _I, [_VP, _VP, _VP, _I, _D, _I, _I, _I, _VP, _VP]),
    ("ls_mlp_create", _I, [_VP, ctypes.POINTER(_VP)]),
    ("ls_mlp_get_params", _I, [_VP, _VP]),
    ("ls_mlp_forward_backward", _I, [_VP, _VP, _VP, _I, _VP, _VP, ctypes.POINTER(ctypes.c_double), _VP]),
    ("ls_mlp_forward", _I, [_VP, _VP, _I, _VP, _VP]),
    ("ls_mlp_adam_step", _I, [_VP, _D, _VP]),
    ("ls_mlp_add_samples", _I, [_VP, _VP, _VP, _I, _VP]),
    ("ls_mlp_num_samples", ctypes.c_long, [_VP]),
    ("ls_mlp_get_samples", _I, [_VP, _VP, _VP]),
    ("ls_mlp_train", _I, [_VP, _I, _I, _D, ctypes.c_uint, _VP, _VP]),
    ("ls_mlp_save", _I, [_VP, ctypes.c_char_p]),
    ("ls_mlp_load", _I, [ctypes.c_char_p, ctypes.POINTER(_VP)]),
    ("ls_mlp_destroy", None, [_VP]),
    ("ls_stencil_fit_learned", _I, [_VP, _VP, ctypes.POINTER(_I), _VP]),
    ("ls_get_learned_info", _I, [_VP, _VP, _VP]),
    ("ls_hbm_copy", _I, [_VP, _VP, ctypes.c_size_t, _VP]),
    ("ls_apply_noalloc", _I, [_VP, _VP, _VP, _I, _I, _VP]),
    ("ls_sparse_factor_host", _I, [_I, _VP, ctypes.c_size_t, _I, ctypes.POINTER(_VP)]),
    ("ls_sparse_solve_host", _I, [_VP, _VP, _I]),
    ("ls_sparse_factor_gpu", _I, [_I, _VP, _I, _VP, ctypes.POINTER(_VP)]),
    ("ls_sparse_solve_gpu", _I, [_VP, _VP, _I, _VP]),
    ("ls_sparse_info", _I, [_VP, ctypes.POINTER(ctypes.c_size_t), ctypes.POINTER(ctypes.c_double)]),
    ("ls_sparse_destroy", None, [_VP]),
    ("ls_plan_fft_size", _I, [_VP]),
    ("ls_plan_set_form", _I, [_VP, _I, _VP]),
    ("ls_plan_tune", _I, [_VP, _I, _I, _VP, _VP]), ("ls_plan_set_tune", _I, [_VP, _I, _I, _I, _I, _I]),
    ("ls_plan_destroy", None, [_VP]),
    # the 2-D variant
    ("ls2_plan_create", _I, [_I, _D, _I, _VP, _VP, ctypes.POINTER(_VP)]),
    ("ls2_apply", _I, [_VP, _VP, _VP, _I, _I, _VP]),
    ("ls2_apply_timed", _I, [_VP, _VP, _VP, _I, _I, _VP, ctypes.POINTER(ctypes.c_double)]),
    ("ls2_rhs_from_incident", _I, [_VP, _VP, _VP, _I, _VP]),
    ("ls2_stencil_fit", _I, [_VP, _VP]),
    ("ls2_get_stencils", _I, [_VP, _VP, _VP, _VP]),
    ("ls2_factor", _I, [_VP, _I, ctypes.POINTER(ctypes.c_double)]),
    ("ls2_factor_gpu", _I, [_VP, _I, _VP, ctypes.POINTER(ctypes.c_double)]),
    ("ls2_precond_apply", _I, [_VP, _VP, _VP, _I, _VP]),
    ("ls2_gmres_solve", _I, [_VP, _VP, _VP, _I, _D, _I, _I, _I, _VP, _VP]),
    ("ls2_plan_fft_size", _I, [_VP]),
    ("ls2_plan_destroy", None, [_VP]),
]


class TuneInfo(ctypes.Structure):
    _fields_ = [("chunk", ctypes.c_int), ("kmul_w", ctypes.c_int), ("ms_per_rhs", ctypes.c_double),
                ("ms_default_per_rhs", ctypes.c_double), ("from_cache", ctypes.c_int), ("n_tried", ctypes.c_int),
                ("half_runs", ctypes.c_int), ("persist", ctypes.c_int)]

    def as_dict(self):
        return {f: getattr(self, f) for f, _ in self._fields_}


class SolveInfo(ctypes.Structure):
    _fields_ = [("iters", ctypes.c_int), ("restarts", ctypes.c_int), ("rel_resid", ctypes.c_double),
                ("t_gpu", ctypes.c_double), ("t_host", ctypes.c_double)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class SparseHost:
    """The host multifrontal solver on its own (host memory only, no GPU needed)."""

    def __init__(self, n: int, rows, host_mem_cap: int = 0, prec: str = "c128"):
        import numpy as np
        lib = load()
        rows = np.ascontiguousarray(rows, dtype=np.complex128)
        if rows.shape != (n ** 3, 3, 27, 3):
            raise ValueError("rows must have shape (n^3, 3, 27, 3)")
        self.n = n
        h = ctypes.c_void_p()
        _check(lib.ls_sparse_factor_host(n, rows.ctypes.data_as(ctypes.c_void_p), host_mem_cap, PREC[prec],
                                         ctypes.byref(h)), "ls_sparse_factor_host")
        self._h = h

    def solve(self, b):
        """x = S^-1 b for b of shape (nrhs, 3, n, n, n) complex128 (host)."""
        import numpy as np
        x = np.array(b, dtype=np.complex128, order="C", copy=True)
        _check(_lib.ls_sparse_solve_host(self._h, x.ctypes.data_as(ctypes.c_void_p), x.shape[0]),
               "ls_sparse_solve_host")
        return x

    def info(self):
        nb, fl = ctypes.c_size_t(), ctypes.c_double()
        _check(_lib.ls_sparse_info(self._h, ctypes.byref(nb), ctypes.byref(fl)), "ls_sparse_info")
        return {"bytes": nb.value, "flops": fl.value}

    def close(self):
        if getattr(self, "_h", None):
            _lib.ls_sparse_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class SparseGpu(SparseHost):
    """The GPU multifrontal solver on its own: rows from the host, factor and
    solves in device memory."""

    def __init__(self, n: int, rows, prec: str = "c128"):
        import numpy as np
        lib = load()
        rows = np.ascontiguousarray(rows, dtype=np.complex128)
        if rows.shape != (n ** 3, 3, 27, 3):
            raise ValueError("rows must have shape (n^3, 3, 27, 3)")
        self.n = n
        h = ctypes.c_void_p()
        _check(lib.ls_sparse_factor_gpu(n, rows.ctypes.data_as(ctypes.c_void_p), PREC[prec], _stream(),
                                        ctypes.byref(h)), "ls_sparse_factor_gpu")
        self._h = h

    def solve(self, b):
        """x = S^-1 b in place for a device tensor b (nrhs, 3, n, n, n) complex128."""
        import torch
        _field(b, torch.complex128, self.n, "b")
        _check(_lib.ls_sparse_solve_gpu(self._h, _ptr(b), b.shape[0], _stream()), "ls_sparse_solve_gpu")
        return b


MLP_NPARAM = 250324


def _fp(a):
    return a.ctypes.data_as(ctypes.c_void_p)


class Mlp:
    """The stencil-prediction network on the GPU (see include/ls.h)."""

    def __init__(self, params=None, path: str | None = None):
        import numpy as np
        lib = load()
        h = ctypes.c_void_p()
        if path is not None:
            _check(lib.ls_mlp_load(path.encode(), ctypes.byref(h)), "ls_mlp_load")
        else:
            p = np.ascontiguousarray(params, dtype=np.float32)
            if p.size != MLP_NPARAM:
                raise ValueError(f"need {MLP_NPARAM} parameters")
            _check(lib.ls_mlp_create(_fp(p), ctypes.byref(h)), "ls_mlp_create")
        self._h = h

    @staticmethod
    def flat(params) -> "np.ndarray":
        """Flat float32 layout from a dict W1, b1, W2, b2, W3, b3 (arrays shaped (in, out))."""
        import numpy as np
        return np.concatenate([np.asarray(params[k], dtype=np.float64).reshape(-1)
                               for k in ("W1", "b1", "W2", "b2", "W3", "b3")]).astype(np.float32)

    @staticmethod
    def unflat(v) -> dict:
        import numpy as np
        v = np.asarray(v, dtype=np.float64)
        out, o = {}, 0
        for k, shp in (("W1", (250, 256)), ("b1", (256,)), ("W2", (256, 256)), ("b2", (256,)),
                       ("W3", (256, 468)), ("b3", (468,))):
            cnt = int(np.prod(shp))
            out[k] = v[o:o + cnt].reshape(shp)
            o += cnt
        return out

    def params(self):
        import numpy as np
        p = np.zeros(MLP_NPARAM, np.float32)
        _check(_lib.ls_mlp_get_params(self._h, _fp(p)), "ls_mlp_get_params")
        return p

    def forward_backward(self, x, t):
        """(y (B, 468), flat grad, loss) for host x (B, 250), t (B, 468)."""
        import numpy as np
        x = np.ascontiguousarray(x, dtype=np.float32)
        t = np.ascontiguousarray(t, dtype=np.float32)
        B = x.shape[0]
        y = np.zeros((B, 468), np.float32)
        g = np.zeros(MLP_NPARAM, np.float32)
        loss = ctypes.c_double()
        _check(_lib.ls_mlp_forward_backward(self._h, _fp(x), _fp(t), B, _fp(y), _fp(g), ctypes.byref(loss),
                                            _stream()), "ls_mlp_forward_backward")
        return y, g, loss.value

    def forward(self, x):
        """y (B, 468) for host x (B, 250): the inference the learned fit runs."""
        import numpy as np
        x = np.ascontiguousarray(x, dtype=np.float32)
        y = np.zeros((x.shape[0], 468), np.float32)
        _check(_lib.ls_mlp_forward(self._h, _fp(x), x.shape[0], _fp(y), _stream()), "ls_mlp_forward")
        return y

    def adam_step(self, lr: float):
        _check(_lib.ls_mlp_adam_step(self._h, float(lr), _stream()), "ls_mlp_adam_step")

    def add_samples(self, plan: "Plan", points):
        import numpy as np
        pts = np.ascontiguousarray(points, dtype=np.int32)
        _check(_lib.ls_mlp_add_samples(self._h, plan._h, _fp(pts), len(pts), _stream()), "ls_mlp_add_samples")

    def num_samples(self) -> int:
        return int(_lib.ls_mlp_num_samples(self._h))

    def samples(self):
        import numpy as np
        N = self.num_samples()
        x = np.zeros((N, 256), np.float32)
        t = np.zeros((N, 468), np.float32)
        _check(_lib.ls_mlp_get_samples(self._h, _fp(x), _fp(t)), "ls_mlp_get_samples")
        return x, t

    def train(self, steps: int, batch: int = 4096, lr: float = 1e-3, seed: int = 0):
        import numpy as np
        loss = np.zeros(steps, np.float64)
        _check(_lib.ls_mlp_train(self._h, steps, batch, float(lr), seed, _fp(loss), _stream()), "ls_mlp_train")
        return loss

    def save(self, path: str):
        _check(_lib.ls_mlp_save(self._h, path.encode()), "ls_mlp_save")

    def close(self):
        if getattr(self, "_h", None):
            _lib.ls_mlp_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


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


def hbm_copy(dst, src, nbytes: int):
    """Streaming device copy of nbytes from src to dst (device tensors) on the current stream."""
    load()
    _check(_lib.ls_hbm_copy(ctypes.c_void_p(dst.data_ptr()), ctypes.c_void_p(src.data_ptr()), nbytes, _stream()),
           "ls_hbm_copy")


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

    def apply_noalloc(self, x, y, prec: str = "c128"):
        """ls_apply_noalloc: the apply with its intermediates in the library's fixed
        device array (no allocation in the call); y must be given."""
        import torch
        dt = torch.complex64 if prec == "c64" else torch.complex128
        _field(x, dt, self.n, "x")
        _field(y, dt, self.n, "y")
        _check(_lib.ls_apply_noalloc(self._h, _ptr(x), _ptr(y), x.shape[0], PREC[prec], _stream()),
               "ls_apply_noalloc")
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

    def stencil_fit(self, mode: int = 0):
        """Class stencils, beta and the rows S on the GPU (Section 3.1, 3.2); mode 1: per point."""
        _check(_lib.ls_stencil_fit(self._h, mode, _stream()), "ls_stencil_fit")

    def stencil_fit_learned(self, mlp: Mlp) -> int:
        """Learned fit with exact fallback; returns the number of fallback points."""
        nf = ctypes.c_int()
        _check(_lib.ls_stencil_fit_learned(self._h, mlp._h, ctypes.byref(nf), _stream()), "ls_stencil_fit_learned")
        return nf.value

    def learned_info(self):
        """(accept (n^3,) int32: 1 accepted, 0 fell back, -1 boundary; ratio (n^3,) float64)."""
        import numpy as np
        acc = np.zeros(self.n ** 3, np.int32)
        rat = np.zeros(self.n ** 3, np.float64)
        _check(_lib.ls_get_learned_info(self._h, acc.ctypes.data_as(ctypes.c_void_p),
                                        rat.ctypes.data_as(ctypes.c_void_p)), "ls_get_learned_info")
        return acc, rat

    def class_stencils(self, gram: bool = False):
        """(alpha, beta, eig[, gram]): alpha, beta (27, 81, 3) complex128; eig (27, 3);
        gram (27, 81, 81) complex128 when asked for."""
        import numpy as np
        al = np.zeros((27, 81, 3), np.complex128)
        be = np.zeros((27, 81, 3), np.complex128)
        ev = np.zeros((27, 3), np.float64)
        gr = np.zeros((27, 81, 81), np.complex128) if gram else None
        _check(_lib.ls_get_class_stencils(self._h, al.ctypes.data_as(ctypes.c_void_p),
                                          be.ctypes.data_as(ctypes.c_void_p),
                                          ev.ctypes.data_as(ctypes.c_void_p),
                                          gr.ctypes.data_as(ctypes.c_void_p) if gram else None),
               "ls_get_class_stencils")
        return (al, be, ev, gr) if gram else (al, be, ev)

    def point_stencils(self):
        """(alpha (n^3, 81, 3) complex128, eig (n^3, 3)) after a per-point fit."""
        import numpy as np
        al = np.zeros((self.n ** 3, 81, 3), np.complex128)
        ev = np.zeros((self.n ** 3, 3), np.float64)
        _check(_lib.ls_get_point_stencils(self._h, al.ctypes.data_as(ctypes.c_void_p),
                                          ev.ctypes.data_as(ctypes.c_void_p)), "ls_get_point_stencils")
        return al, ev

    def rows(self):
        """Assembled rows S, (n^3, 3, 27, 3) complex128."""
        import numpy as np
        r = np.zeros((self.n ** 3, 3, 27, 3), np.complex128)
        _check(_lib.ls_get_rows(self._h, r.ctypes.data_as(ctypes.c_void_p)), "ls_get_rows")
        return r

    def set_form(self, form: str):
        """Operator form of the apply: "dyadic" (the default) or "paper" (Section 2's own form)."""
        _check(_lib.ls_plan_set_form(self._h, {"dyadic": 0, "paper": 1}[form], _stream()), "ls_plan_set_form")

    def factor_gpu(self, prec: str = "c128"):
        """GPU multifrontal LU of S (complex128 or complex64 factor); returns seconds."""
        t = ctypes.c_double()
        _check(_lib.ls_factor_gpu(self._h, PREC[prec], _stream(), ctypes.byref(t)), "ls_factor_gpu")
        return t.value

    def factor(self, prec: str = "c128"):
        """Host multifrontal LU of S (complex128 or complex64 factor); returns seconds."""
        t = ctypes.c_double()
        _check(_lib.ls_factor_prec(self._h, PREC[prec], ctypes.byref(t)), "ls_factor_prec")
        return t.value

    def precond(self, v, z=None):
        """z = S^-1 Q v (complex128 device fields)."""
        import torch
        _field(v, torch.complex128, self.n, "v")
        if z is None:
            z = torch.empty_like(v)
        _check(_lib.ls_precond_apply(self._h, _ptr(v), _ptr(z), v.shape[0], _stream()), "ls_precond_apply")
        return z

    def solve(self, g, tol: float = 1e-8, restart: int = 30, maxit: int = 500, prec: str = "c128",
              x=None, check: bool = True):
        """FGMRES solve A x = g; returns (x, [info dict per rhs], status)."""
        import torch
        _field(g, torch.complex128, self.n, "g")
        if x is None:
            x = torch.empty_like(g)
        nr = g.shape[0]
        infos = (SolveInfo * nr)()
        st = _lib.ls_gmres_solve(self._h, _ptr(g), _ptr(x), nr, float(tol), restart, maxit, PREC[prec],
                                 ctypes.cast(infos, ctypes.c_void_p), _stream())
        if check and st not in (0, -4):
            _check(st, "ls_gmres_solve")
        return x, [i.as_dict() for i in infos], st

    def tune(self, nrhs: int, prec: str = "c64") -> dict:
        """Autotune the batched apply (cache: the plan's tune_cache file)."""
        info = TuneInfo()
        _check(_lib.ls_plan_tune(self._h, nrhs, PREC[prec], _stream(), ctypes.byref(info)), "ls_plan_tune")
        return info.as_dict()

    def set_tune(self, prec: str, chunk: int = 0, kmul_w: int = 0, half_runs: int = 0, persist: int = 0):
        _check(_lib.ls_plan_set_tune(self._h, PREC[prec], chunk, kmul_w, half_runs, persist), "ls_plan_set_tune")

    def rhs_from_incident(self, Ei, g=None):
        """g = -K * (m E^i) (right-hand side of Eq. (4)), complex128."""
        import torch
        _field(Ei, torch.complex128, self.n, "Ei")
        if g is None:
            g = torch.empty_like(Ei)
        _check(_lib.ls_rhs_from_incident(self._h, _ptr(Ei), _ptr(g), Ei.shape[0], _stream()),
               "ls_rhs_from_incident")
        return g


def _field2(t, dtype, n, name):
    if not t.is_cuda or t.dtype != dtype or not t.is_contiguous():
        raise ValueError(f"{name}: need a contiguous CUDA tensor of {dtype}")
    if t.dim() != 4 or tuple(t.shape[1:]) != (2, n, n):
        raise ValueError(f"{name}: shape must be (nrhs, 2, {n}, {n}), got {tuple(t.shape)}")
    return t


class Plan2:
    """A plan of the 2-D variant: contrast, p, symbol and workspaces on the GPU."""

    def __init__(self, n: int, k: float, m, max_rhs: int = 1):
        import torch
        lib = load()
        if m.dtype != torch.complex128 or not m.is_cuda or tuple(m.shape) != (n, n):
            raise ValueError("m must be a (n, n) complex128 CUDA tensor")
        m = m.contiguous()
        self.n, self.k, self.max_rhs = n, float(k), max_rhs
        h = ctypes.c_void_p()
        _check(lib.ls2_plan_create(n, float(k), max_rhs, _ptr(m), _stream(), ctypes.byref(h)), "ls2_plan_create")
        self._h = h
        self.P = lib.ls2_plan_fft_size(h)

    def close(self):
        if getattr(self, "_h", None):
            _lib.ls2_plan_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def apply(self, x, y=None, prec: str = "c128"):
        """y = A x; x complex128 (c128, mixed) or complex64 (c64), shape (nrhs, 2, n, n)."""
        import torch
        dt = torch.complex64 if prec == "c64" else torch.complex128
        _field2(x, dt, self.n, "x")
        if y is None:
            y = torch.empty_like(x)
        _field2(y, dt, self.n, "y")
        _check(_lib.ls2_apply(self._h, _ptr(x), _ptr(y), x.shape[0], PREC[prec], _stream()), "ls2_apply")
        return y

    def apply_timed(self, x, y, prec: str = "c128"):
        """ls2_apply_timed: the three pass times in ms."""
        import torch
        dt = torch.complex64 if prec == "c64" else torch.complex128
        _field2(x, dt, self.n, "x")
        _field2(y, dt, self.n, "y")
        ms = (ctypes.c_double * 3)()
        _check(_lib.ls2_apply_timed(self._h, _ptr(x), _ptr(y), x.shape[0], PREC[prec], _stream(), ms),
               "ls2_apply_timed")
        return list(ms)

    def rhs_from_incident(self, Ei, g=None):
        import torch
        _field2(Ei, torch.complex128, self.n, "Ei")
        if g is None:
            g = torch.empty_like(Ei)
        _check(_lib.ls2_rhs_from_incident(self._h, _ptr(Ei), _ptr(g), Ei.shape[0], _stream()),
               "ls2_rhs_from_incident")
        return g

    def stencil_fit(self):
        _check(_lib.ls2_stencil_fit(self._h, _stream()), "ls2_stencil_fit")

    def stencils(self):
        """(alpha [9][18][2], beta [9][27][2], eig [9][18]) as numpy arrays."""
        import numpy as np
        a = np.zeros((9, 18, 2), dtype=np.complex128)
        b = np.zeros((9, 27, 2), dtype=np.complex128)
        e = np.zeros((9, 18), dtype=np.float64)
        _check(_lib.ls2_get_stencils(self._h, a.ctypes.data_as(_VP), b.ctypes.data_as(_VP), e.ctypes.data_as(_VP)),
               "ls2_get_stencils")
        return a, b, e

    def factor(self, prec: str = "c128") -> float:
        t = ctypes.c_double()
        _check(_lib.ls2_factor(self._h, PREC[prec], ctypes.byref(t)), "ls2_factor")
        return t.value

    def factor_gpu(self, prec: str = "c128") -> float:
        t = ctypes.c_double()
        _check(_lib.ls2_factor_gpu(self._h, PREC[prec], _stream(), ctypes.byref(t)), "ls2_factor_gpu")
        return t.value

    def precond(self, v, z=None):
        import torch
        _field2(v, torch.complex128, self.n, "v")
        if z is None:
            z = torch.empty_like(v)
        _check(_lib.ls2_precond_apply(self._h, _ptr(v), _ptr(z), v.shape[0], _stream()), "ls2_precond_apply")
        return z

    def solve(self, g, tol: float = 1e-8, restart: int = 30, maxit: int = 500, prec: str = "c128"):
        """FGMRES; returns (x, [info dicts], status)."""
        import torch
        _field2(g, torch.complex128, self.n, "g")
        x = torch.zeros_like(g)
        nr = g.shape[0]
        infos = (SolveInfo * nr)()
        st = _lib.ls2_gmres_solve(self._h, _ptr(g), _ptr(x), nr, float(tol), restart, maxit, PREC[prec],
                                  ctypes.cast(infos, _VP), _stream())
        if st not in (0, -4):
            _check(st, "ls2_gmres_solve")
        out = [dict(iters=i.iters, restarts=i.restarts, rel_resid=i.rel_resid, t_gpu=i.t_gpu, t_host=i.t_host)
               for i in infos]
        return x, out, st
