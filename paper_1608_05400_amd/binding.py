"""ctypes binding of ``libmgwr.so`` (declared in ``include/mgwr.h``).

Argument marshalling only: every step of the solver runs in the HIP library.
Arrays are torch tensors on the GPU (float64, contiguous); torch provides the
device memory and the stream (``torch.cuda.current_stream()``).  There is no
CPU fallback: if the library cannot be loaded, every entry point raises.
"""
from __future__ import annotations

import ctypes
import os
from typing import Optional, Sequence

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libmgwr.so")

MGWR_OK, MGWR_NOT_CONVERGED, MGWR_STAGNATED = 0, 1, 2
MGWR_EINVAL, MGWR_ENOMEM, MGWR_EDEVICE, MGWR_ENONFINITE, MGWR_EDIVERGED = -1, -2, -3, -4, -5
FP64, MIXED_FP32, MIXED_BF16X3, FP64_REFINED = 0, 1, 2, 3
PRECISIONS = {"fp64": FP64, "fp32": MIXED_FP32, "bf16x3": MIXED_BF16X3, "fp64r": FP64_REFINED}
NORM_MAX, NORM_L2 = 0, 1
SMOOTH_INVERSE, SMOOTH_DC, SMOOTH_AUTO = 0, 1, 2
SMOOTHERS = {"inverse": SMOOTH_INVERSE, "dc": SMOOTH_DC, "auto": SMOOTH_AUTO}
STATUS_NAMES = {0: "ok", 1: "not_converged", 2: "stagnated", -1: "einval", -2: "enomem",
                -3: "edevice", -4: "enonfinite", -5: "ediverged"}

EXPORTED = [
    "mgwr_default_options", "mgwr_l1_weights", "mgwr_create", "mgwr_create_ex", "mgwr_destroy",
    "mgwr_set_options", "mgwr_get_options", "mgwr_set_stream", "mgwr_smooth", "mgwr_residual",
    "mgwr_vcycle", "mgwr_solve", "mgwr_toeplitz_apply", "mgwr_get_column", "mgwr_levels",
    "mgwr_batch_create", "mgwr_batch_solve", "mgwr_batch_set_stream", "mgwr_batch_destroy",
    "mgwr_profile_enable", "mgwr_profile_count", "mgwr_profile_get", "mgwr_kernel_name",
    "mgwr_last_error", "mgwr_autotune", "mgwr_get_tuning", "mgwr_batch_autotune",
    "mgwr_batch_get_tuning", "mgwr_batch_profile_enable", "mgwr_batch_profile_count",
    "mgwr_batch_profile_get", "mgwr_fas_solve", "mgwr_fas_solve_batch", "mgwr_set_tuning",
    "mgwr_toeplitz_apply_static",
]


class MgwrError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"{STATUS_NAMES.get(code, code)}: {msg}")
        self.code = code


class Options(ctypes.Structure):
    _fields_ = [("nu1", ctypes.c_int), ("nu2", ctypes.c_int), ("gamma", ctypes.c_int),
                ("maxit", ctypes.c_int), ("norm", ctypes.c_int), ("warm_start", ctypes.c_int),
                ("precision", ctypes.c_int), ("first_colour", ctypes.c_int),
                ("smoother", ctypes.c_int), ("dc_block", ctypes.c_int),
                ("L", ctypes.c_double), ("stall", ctypes.c_double), ("graph", ctypes.c_int),
                ("fft", ctypes.c_int), ("inner_cycles", ctypes.c_int)]


class Tuning(ctypes.Structure):
    _fields_ = [("tuned", ctypes.c_int), ("variant", ctypes.c_int * 2),
                ("split_target", ctypes.c_int * 3), ("levels", ctypes.c_int),
                ("dc_block", ctypes.c_int * 32), ("fft", ctypes.c_int * 32),
                ("ms_default", ctypes.c_double), ("ms_tuned", ctypes.c_double)]

    def as_dict(self):
        return {"tuned": bool(self.tuned), "variant": list(self.variant),
                "split_target": list(self.split_target),
                "dc_block": list(self.dc_block[:self.levels]),
                "fft": list(self.fft[:self.levels]),
                "ms_default": self.ms_default, "ms_tuned": self.ms_tuned}


class KernelRecord(ctypes.Structure):
    _fields_ = [("kernel", ctypes.c_int), ("level", ctypes.c_int), ("M", ctypes.c_int),
                ("P", ctypes.c_int), ("K", ctypes.c_int), ("flops", ctypes.c_double),
                ("ms", ctypes.c_double), ("bytes", ctypes.c_double), ("pass_bytes", ctypes.c_double),
                ("products", ctypes.c_int)]


class Info(ctypes.Structure):
    _fields_ = [("iters", ctypes.c_int), ("status", ctypes.c_int), ("r0", ctypes.c_double),
                ("rk", ctypes.c_double), ("relres", ctypes.c_double),
                ("mean_factor", ctypes.c_double), ("hist", ctypes.c_double * 128)]

    def as_dict(self):
        n = min(self.iters, 127) + 1
        return {"iters": self.iters, "status": STATUS_NAMES.get(self.status, self.status),
                "r0": self.r0, "rk": self.rk, "relres": self.relres,
                "mean_factor": self.mean_factor, "hist": list(self.hist[:n])}


_lib = None


def load(path: str = LIB_PATH):
    """Load the HIP library; build it first only if no build exists."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        from . import build as _build
        _build.build()
    lib = ctypes.CDLL(path)
    P, I, D, VP = ctypes.POINTER, ctypes.c_int, ctypes.c_double, ctypes.c_void_p
    h = ctypes.c_void_p
    lib.mgwr_default_options.argtypes = [P(Options)]
    lib.mgwr_l1_weights.argtypes = [I, D, D, P(D), P(D)]
    lib.mgwr_create.argtypes = [I, I, D, D, I, P(h)]
    lib.mgwr_create_ex.argtypes = [I, I, D, D, I, P(Options), P(h)]
    lib.mgwr_destroy.argtypes = [h]
    lib.mgwr_set_options.argtypes = [h, P(Options)]
    lib.mgwr_get_options.argtypes = [h, P(Options)]
    lib.mgwr_set_stream.argtypes = [h, VP]
    lib.mgwr_smooth.argtypes = [h, VP, VP, VP, I]
    lib.mgwr_residual.argtypes = [h, VP, VP, VP, VP, P(D)]
    lib.mgwr_vcycle.argtypes = [h, VP, VP, VP]
    lib.mgwr_solve.argtypes = [h, VP, VP, VP, D, P(Info)]
    lib.mgwr_toeplitz_apply.argtypes = [h, I, I, VP, I, I, VP, I]
    lib.mgwr_toeplitz_apply_static.argtypes = [h, I, I, VP, I, I, VP, I]
    lib.mgwr_get_column.argtypes = [h, I, P(D)]
    lib.mgwr_levels.argtypes = [h]
    lib.mgwr_batch_create.argtypes = [I, P(I), P(I), P(D), P(D), I, P(Options), P(h)]
    lib.mgwr_batch_solve.argtypes = [h, P(VP), P(VP), P(VP), D, P(Info)]
    lib.mgwr_batch_set_stream.argtypes = [h, VP]
    lib.mgwr_batch_destroy.argtypes = [h]
    lib.mgwr_profile_enable.argtypes = [h, I]
    lib.mgwr_profile_count.argtypes = [h]
    lib.mgwr_profile_get.argtypes = [h, I, P(KernelRecord)]
    lib.mgwr_autotune.argtypes = [h]
    lib.mgwr_get_tuning.argtypes = [h, P(Tuning)]
    lib.mgwr_set_tuning.argtypes = [h, P(Tuning)]
    lib.mgwr_batch_autotune.argtypes = [h]
    lib.mgwr_batch_get_tuning.argtypes = [h, I, P(Tuning)]
    lib.mgwr_batch_profile_enable.argtypes = [h, I]
    lib.mgwr_batch_profile_count.argtypes = [h]
    lib.mgwr_batch_profile_get.argtypes = [h, I, P(KernelRecord)]
    lib.mgwr_fas_solve.argtypes = [I, I, D, D, D, D, I, I, I, VP, VP, D, I, VP, P(Info)]
    lib.mgwr_fas_solve_batch.argtypes = [I, I, I, P(D), D, D, D, I, I, I, P(VP), P(VP), D, I, VP, P(Info)]
    lib.mgwr_kernel_name.argtypes = [I]
    lib.mgwr_kernel_name.restype = ctypes.c_char_p
    lib.mgwr_last_error.restype = ctypes.c_char_p
    _lib = lib
    return lib


def last_error() -> str:
    return load().mgwr_last_error().decode()


def _check(rc, allow_positive=True):
    if rc < 0 or (rc > 0 and not allow_positive):
        raise MgwrError(rc, last_error())
    return rc


def _option_value(k, v):
    if k == "precision" and isinstance(v, str):
        return PRECISIONS[v]
    if k == "norm" and isinstance(v, str):
        return {"max": NORM_MAX, "l2": NORM_L2}[v]
    if k == "smoother" and isinstance(v, str):
        return SMOOTHERS[v]
    if isinstance(v, bool):
        return int(v)
    return v


def default_options(**kw) -> Options:
    o = Options()
    load().mgwr_default_options(ctypes.byref(o))
    for k, v in kw.items():
        if not hasattr(o, k):
            raise TypeError(f"unknown option {k}")
        setattr(o, k, _option_value(k, v))
    return o


def _records(count, get, handle):
    n = _check(count(handle))
    out = []
    rec = KernelRecord()
    for i in range(n):
        _check(get(handle, i, ctypes.byref(rec)), False)
        out.append({"kernel": rec.kernel, "name": kernel_name(rec.kernel), "level": rec.level,
                    "M": rec.M, "P": rec.P, "K": rec.K, "flops": rec.flops, "ms": rec.ms,
                    "bytes": rec.bytes, "pass_bytes": rec.pass_bytes, "products": rec.products})
    return out


def l1_weights(M: int, alpha: float, T: float = 1.0):
    """Host-side L1 weights (c, r[0..M-1]) computed by the library."""
    import numpy as np
    r = np.zeros(M)
    c = ctypes.c_double()
    _check(load().mgwr_l1_weights(M, alpha, T, ctypes.byref(c),
                                  r.ctypes.data_as(ctypes.POINTER(ctypes.c_double))), False)
    return c.value, r


def fas_solve(f, u, alpha: float, c: float = 1.0, q: float = 1.0, nu1: int = 0, nu2: int = 1,
              first_colour: int = 1, tol: float = 1e-10, maxit: int = 60, T: float = 1.0,
              raise_on_error: bool = True):
    """Waveform relaxation FAS for the nonlinear problem of Section 7
    (mgwr_fas_solve); f, u: device FP64 [M, N] tensors, u receives the
    solution.  Returns the info dict with the return code under "rc"."""
    M, N = u.shape
    info = Info()
    rc = load().mgwr_fas_solve(N, M, alpha, T, c, q, nu1, nu2, first_colour, _ptr(f, "f", (M, N)),
                               _ptr(u, "u", (M, N)), tol, maxit, _stream(), ctypes.byref(info))
    if rc < 0 and raise_on_error:
        raise MgwrError(rc, last_error())
    d = info.as_dict()
    d["rc"] = rc
    return d


def fas_solve_batch(fs, us, alphas, c: float = 1.0, q: float = 1.0, nu1: int = 0, nu2: int = 1,
                    first_colour: int = 1, tol: float = 1e-10, maxit: int = 60, T: float = 1.0,
                    raise_on_error: bool = True):
    """Several problems of the nonlinear problem of Section 7 with the same
    shape (mgwr_fas_solve_batch); returns (rc, [info dicts])."""
    n = len(us)
    M, N = us[0].shape
    fp = (ctypes.c_void_p * n)(*[_ptr(f, "f", (M, N)) for f in fs])
    up = (ctypes.c_void_p * n)(*[_ptr(u, "u", (M, N)) for u in us])
    infos = (Info * n)()
    rc = load().mgwr_fas_solve_batch(n, N, M, (ctypes.c_double * n)(*alphas), T, c, q, nu1, nu2, first_colour,
                                     fp, up, tol, maxit, _stream(), infos)
    if rc < 0 and raise_on_error:
        raise MgwrError(rc, last_error())
    return rc, [i.as_dict() for i in infos]


def kernel_name(kernel: int) -> str:
    return load().mgwr_kernel_name(kernel).decode()


def _ptr(t, name, shape=None, allow_none=False):
    import torch
    if t is None:
        if allow_none:
            return None
        raise ValueError(f"{name} is required")
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError(f"{name} must be a CUDA (HIP) torch tensor")
    if t.dtype != torch.float64:
        raise TypeError(f"{name} must be float64")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    if shape is not None and tuple(t.shape) != tuple(shape):
        raise ValueError(f"{name} has shape {tuple(t.shape)}, expected {tuple(shape)}")
    return ctypes.c_void_p(t.data_ptr())


def _stream():
    import torch
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


class Solver:
    """Handle of one problem: N interior points per dimension (2^k - 1), M time
    steps, fractional order alpha, final time T, dims in {1, 2}."""

    def __init__(self, N: int, M: int, alpha: float, T: float = 1.0, dims: int = 1, **opts):
        self.N, self.M, self.alpha, self.T, self.dims = N, M, alpha, T, dims
        self._lib = load()
        self._h = ctypes.c_void_p()
        o = default_options(**opts)
        _check(self._lib.mgwr_create_ex(N, M, alpha, T, dims, ctypes.byref(o), ctypes.byref(self._h)),
               False)

    @property
    def grid_shape(self):
        return (self.M, self.N) if self.dims == 1 else (self.M, self.N, self.N)

    @property
    def ic_shape(self):
        return self.grid_shape[1:]

    def close(self):
        if self._h:
            self._lib.mgwr_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()

    def options(self) -> Options:
        o = Options()
        _check(self._lib.mgwr_get_options(self._h, ctypes.byref(o)))
        return o

    def set_options(self, **kw):
        o = self.options()
        for k, v in kw.items():
            if not hasattr(o, k):
                raise TypeError(f"unknown option {k}")
            setattr(o, k, _option_value(k, v))
        _check(self._lib.mgwr_set_options(self._h, ctypes.byref(o)), False)

    def autotune(self):
        """Time tile shapes (and D&C base blocks) on the handle's own buffers
        and keep the fastest; returns the choice."""
        self._bind_stream()
        _check(self._lib.mgwr_autotune(self._h), False)
        return self.tuning()

    def tuning(self):
        t = Tuning()
        _check(self._lib.mgwr_get_tuning(self._h, ctypes.byref(t)), False)
        return t.as_dict()

    def set_tuning(self, d):
        """Apply a tuning dict from tuning() (mgwr_set_tuning)."""
        t = Tuning()
        t.tuned = 1
        t.variant[:] = list(d["variant"])
        t.split_target[:] = list(d["split_target"])
        t.levels = len(d["fft"])
        if len(d["dc_block"]) != t.levels or t.levels > 32:
            raise ValueError("dc_block and fft must have one entry per level")
        for l in range(t.levels):
            t.dc_block[l] = int(d["dc_block"][l])
            t.fft[l] = int(d["fft"][l])
        t.ms_default = float(d.get("ms_default", 0.0))
        t.ms_tuned = float(d.get("ms_tuned", 0.0))
        _check(self._lib.mgwr_set_tuning(self._h, ctypes.byref(t)), False)

    def save_tuning(self, path):
        """Write the handle's tuning as JSON (to reuse in a later process)."""
        import json
        with open(path, "w") as fh:
            json.dump(self.tuning(), fh)

    def load_tuning(self, path):
        """Apply a tuning written by save_tuning for a handle of the same shape."""
        import json
        with open(path) as fh:
            self.set_tuning(json.load(fh))

    def levels(self) -> int:
        return _check(self._lib.mgwr_levels(self._h))

    def _bind_stream(self):
        _check(self._lib.mgwr_set_stream(self._h, _stream()))

    def smooth(self, f, u, g=None, sweeps=1):
        self._bind_stream()
        _check(self._lib.mgwr_smooth(self._h, _ptr(f, "f", self.grid_shape),
                                     _ptr(g, "g", self.ic_shape, True),
                                     _ptr(u, "u", self.grid_shape), sweeps), False)
        return u

    def residual(self, f, u, g=None, r=None, norms=False):
        import torch
        if r is None:
            r = torch.empty_like(u)
        self._bind_stream()
        nrm = (ctypes.c_double * 2)()
        _check(self._lib.mgwr_residual(self._h, _ptr(f, "f", self.grid_shape),
                                       _ptr(g, "g", self.ic_shape, True),
                                       _ptr(u, "u", self.grid_shape), _ptr(r, "r", self.grid_shape),
                                       nrm if norms else None), False)
        return (r, (nrm[0], nrm[1])) if norms else r

    def vcycle(self, f, u, g=None):
        self._bind_stream()
        _check(self._lib.mgwr_vcycle(self._h, _ptr(f, "f", self.grid_shape),
                                     _ptr(g, "g", self.ic_shape, True),
                                     _ptr(u, "u", self.grid_shape)), False)
        return u

    def solve(self, f, u, g=None, tol=1e-10, raise_on_error=True):
        self._bind_stream()
        info = Info()
        rc = self._lib.mgwr_solve(self._h, _ptr(f, "f", self.grid_shape),
                                  _ptr(g, "g", self.ic_shape, True), _ptr(u, "u", self.grid_shape),
                                  tol, ctypes.byref(info))
        if rc < 0 and raise_on_error:
            raise MgwrError(rc, last_error())
        d = info.as_dict()
        d["rc"] = rc
        return d

    def toeplitz_apply(self, B, which=-1, precision=FP64, C=None):
        import torch
        if isinstance(precision, str):
            precision = PRECISIONS[precision]
        if B.dim() != 2 or B.shape[0] != self.M:
            raise ValueError("B must be [M, P]")
        if C is None:
            C = torch.empty_like(B)
        self._bind_stream()
        P = B.shape[1]
        _check(self._lib.mgwr_toeplitz_apply(self._h, which, precision, _ptr(B, "B"), P, P,
                                             _ptr(C, "C"), P), False)
        return C

    def toeplitz_apply_static(self, B, which=-1, precision=FP64, C=None):
        """toeplitz_apply through the allocation-free entry point
        (mgwr_toeplitz_apply_static; C must be given by callers that cannot
        allocate)."""
        import torch
        if isinstance(precision, str):
            precision = PRECISIONS[precision]
        if B.dim() != 2 or B.shape[0] != self.M:
            raise ValueError("B must be [M, P]")
        if C is None:
            C = torch.empty_like(B)
        self._bind_stream()
        P = B.shape[1]
        _check(self._lib.mgwr_toeplitz_apply_static(self._h, which, precision, _ptr(B, "B"), P, P,
                                                    _ptr(C, "C"), P), False)
        return C

    def profile(self, on=True):
        """Start (clearing old records) or stop per-launch timing of the products."""
        _check(self._lib.mgwr_profile_enable(self._h, 1 if on else 0), False)

    def profile_records(self):
        return _records(self._lib.mgwr_profile_count, self._lib.mgwr_profile_get, self._h)

    def column(self, which=-1):
        import numpy as np
        out = np.zeros(self.M)
        _check(self._lib.mgwr_get_column(self._h, which,
                                         out.ctypes.data_as(ctypes.POINTER(ctypes.c_double))), False)
        return out


class Batch:
    """Many independent problems of uneven (N, M, alpha) sharing dims/options."""

    def __init__(self, Ns: Sequence[int], Ms: Sequence[int], alphas: Sequence[float],
                 Ts: Optional[Sequence[float]] = None, dims: int = 1, **opts):
        self._lib = load()
        n = len(Ns)
        Ts = Ts if Ts is not None else [1.0] * n
        self.Ns, self.Ms, self.dims = list(Ns), list(Ms), dims
        self._b = ctypes.c_void_p()
        o = default_options(**opts)
        _check(self._lib.mgwr_batch_create(
            n, (ctypes.c_int * n)(*Ns), (ctypes.c_int * n)(*Ms), (ctypes.c_double * n)(*alphas),
            (ctypes.c_double * n)(*Ts), dims, ctypes.byref(o), ctypes.byref(self._b)), False)

    def close(self):
        if self._b:
            self._lib.mgwr_batch_destroy(self._b)
            self._b = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def grid_shape(self, i):
        N, M = self.Ns[i], self.Ms[i]
        return (M, N) if self.dims == 1 else (M, N, N)

    def solve(self, fs, us, gs=None, tol=1e-10, raise_on_error=True):
        n = len(self.Ns)
        if len(fs) != n or len(us) != n or (gs is not None and len(gs) != n):
            raise ValueError(f"need {n} right-hand sides and iterates")
        fp = (ctypes.c_void_p * n)(*[_ptr(f, "f", self.grid_shape(i)).value for i, f in enumerate(fs)])
        up = (ctypes.c_void_p * n)(*[_ptr(u, "u", self.grid_shape(i)).value for i, u in enumerate(us)])
        gp = None
        if gs is not None:
            gp = (ctypes.c_void_p * n)(*[(_ptr(g, "g", self.grid_shape(i)[1:]).value
                                          if g is not None else None) for i, g in enumerate(gs)])
        infos = (Info * n)()
        _check(self._lib.mgwr_batch_set_stream(self._b, _stream()))
        rc = self._lib.mgwr_batch_solve(self._b, fp, gp, up, tol, infos)
        if rc < 0 and raise_on_error:
            raise MgwrError(rc, last_error())
        return rc, [i.as_dict() for i in infos]

    def autotune(self):
        _check(self._lib.mgwr_batch_set_stream(self._b, _stream()))
        _check(self._lib.mgwr_batch_autotune(self._b), False)
        return self.tuning(0)

    def tuning(self, i=0):
        t = Tuning()
        _check(self._lib.mgwr_batch_get_tuning(self._b, i, ctypes.byref(t)), False)
        return t.as_dict()

    def profile(self, on=True):
        _check(self._lib.mgwr_batch_profile_enable(self._b, 1 if on else 0), False)

    def profile_records(self):
        return _records(self._lib.mgwr_batch_profile_count, self._lib.mgwr_batch_profile_get, self._b)
