"""CPU FP64 oracle for multigrid waveform relaxation (MGWR) on the
time-fractional heat equation (Gaspar & Rodrigo, arXiv:1608.05400).

TEST INFRASTRUCTURE ONLY.  Only ``tests/``, ``__graft_entry__.smoke()`` and
the CPU-baseline leg of ``bench.py`` import this package.  It shares no code
with the GPU library (``paper_1608_05400_amd``) and never imports it.

The arithmetic lives in ``mgwr_oracle.c`` (plain C, FP64, compiled with gcc);
this module only builds it and marshals NumPy arrays.  Array conventions
follow the C file: grid functions are ``[M, N]`` (1D) or ``[M, N, N]`` (2D,
x fastest) with row ``m`` holding time level ``t_{m+1}``.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "mgwr_oracle.c")
# MGWR_ORACLE_LIB selects another build of the same source (the sanitizer
# test loads one built with AddressSanitizer and UBSan)
_LIB = os.environ.get("MGWR_ORACLE_LIB") or os.path.join(_HERE, "libmgwr_oracle.so")
_lib = None

_D = ctypes.POINTER(ctypes.c_double)
_I = ctypes.POINTER(ctypes.c_int)


def build(force: bool = True) -> str:
    """Compile the oracle with gcc into ``oracle/libmgwr_oracle.so``."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp"
        cmd = ["gcc", "-O3", "-march=x86-64-v3", "-fopenmp", "-fPIC", "-shared",
               "-std=gnu11", "-o", tmp, _SRC, "-lm"]
        subprocess.run(cmd, check=True)
        os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build(force=True)
        lib = ctypes.CDLL(_LIB)
        dd, ii = ctypes.c_double, ctypes.c_int
        lib.orc_l1_coeffs.argtypes = [ii, dd, dd, _D, _D, _D]
        lib.orc_residual.argtypes = [ii, ii, ii, dd, dd, dd, _D, _D, _D, _D]
        lib.orc_half_sweep.argtypes = [ii, ii, ii, dd, dd, dd, ii, _D, _D, _D]
        lib.orc_restrict.argtypes = [ii, ii, ii, _D, _D]
        lib.orc_prolong_add.argtypes = [ii, ii, ii, _D, _D]
        lib.orc_vcycle.argtypes = [ii, ii, ii, dd, dd, dd, ii, ii, ii, ii, _D, _D, _D]
        lib.orc_mg_solve.argtypes = [ii, ii, ii, dd, dd, dd, ii, ii, ii, ii, ii, dd, ii, ii,
                                     _D, _D, _D, _D]
        lib.orc_mg_solve.restype = ii
        lib.orc_direct_solve.argtypes = [ii, ii, ii, dd, dd, dd, _D, _D, _D, ii]
        lib.orc_modal_solve.argtypes = [ii, ii, ii, dd, dd, dd, ii, _I, _I, _D, _D, _D]
        lib.orc_modal_eval.argtypes = [ii, ii, ii, dd, ii, _I, _I, _D, ii, _I, _D]
        lib.orc_mittag_leffler.argtypes = [dd, ii, _D, _D]
        lib.orc_nl_solve.argtypes = [ii, ii, dd, dd, dd, dd, ii, ii, ii, dd, ii, _D, _D, _D]
        lib.orc_nl_solve.restype = ii
        lib.orc_max_threads.restype = ii
        _lib = lib
    return _lib


def _dp(a):
    return None if a is None else a.ctypes.data_as(_D)


def _ip(a):
    return None if a is None else a.ctypes.data_as(_I)


def _f64(a):
    return None if a is None else np.ascontiguousarray(a, dtype=np.float64)


def _npts(dims, N):
    return N if dims == 1 else N * N


def l1_coeffs(M: int, alpha: float, T: float = 1.0):
    """Return (c, d[0..M], r[1..M]) of the L1 scheme (Section 2; Section 5)."""
    d = np.zeros(M + 1)
    r = np.zeros(M)
    c = ctypes.c_double()
    _load().orc_l1_coeffs(M, alpha, T, ctypes.byref(c), _dp(d), _dp(r))
    return c.value, d, r


def residual(dims, N, M, alpha, f, u, g=None, T=1.0, L=1.0):
    """R = f + c d_m g - T_M u - A_h u (Section 2 / Section 6)."""
    f, u, g = _f64(f), _f64(u), _f64(g)
    R = np.empty_like(f)
    _load().orc_residual(dims, N, M, alpha, T, L, _dp(f), _dp(g), _dp(u), _dp(R))
    return R


def half_sweep(dims, N, M, alpha, colour, f, u, g=None, T=1.0, L=1.0):
    """One red (colour 0) or black (colour 1) waveform-relaxation half-sweep."""
    f, g = _f64(f), _f64(g)
    u = np.array(u, dtype=np.float64, copy=True, order="C")
    _load().orc_half_sweep(dims, N, M, alpha, T, L, colour, _dp(f), _dp(g), _dp(u))
    return u


def restrict(dims, Nf, M, rf):
    rf = _f64(rf)
    Nc = (Nf - 1) // 2
    shape = (M, Nc) if dims == 1 else (M, Nc, Nc)
    rc = np.empty(shape)
    _load().orc_restrict(dims, Nf, M, _dp(rf), _dp(rc))
    return rc


def prolong_add(dims, Nc, M, ec, uf):
    ec = _f64(ec)
    uf = np.array(uf, dtype=np.float64, copy=True, order="C")
    _load().orc_prolong_add(dims, Nc, M, _dp(ec), _dp(uf))
    return uf


def vcycle(dims, N, M, alpha, f, u, g=None, nu1=1, nu2=1, gamma=1, first=0, T=1.0, L=1.0):
    """One cycle of Algorithm 1; ``first`` is the colour relaxed first."""
    f, g = _f64(f), _f64(g)
    u = np.array(u, dtype=np.float64, copy=True, order="C")
    _load().orc_vcycle(dims, N, M, alpha, T, L, nu1, nu2, gamma, first, _dp(f), _dp(g), _dp(u))
    return u


def mg_solve(dims, N, M, alpha, f, g=None, nu1=1, nu2=1, gamma=1, first=0, norm=0, tol=1e-10,
             maxit=100, u0=None, T=1.0, L=1.0):
    """MGWR iteration from u^0 = g (or ``u0`` if given).  Returns (u, hist)."""
    f, g = _f64(f), _f64(g)
    warm = 0
    if u0 is not None:
        u = np.array(u0, dtype=np.float64, copy=True, order="C")
        warm = 1
    else:
        u = np.empty_like(f)
    hist = np.zeros(maxit + 1)
    its = _load().orc_mg_solve(dims, N, M, alpha, T, L, nu1, nu2, gamma, first, norm, tol, maxit,
                               warm, _dp(f), _dp(g), _dp(u), _dp(hist))
    return u, hist[: its + 1].copy()


def direct_solve(dims, N, M, alpha, f, g=None, T=1.0, L=1.0, Mstop=0):
    """Exact discrete solution by sequential time stepping (first Mstop levels)."""
    f, g = _f64(f), _f64(g)
    u = np.zeros_like(f)
    _load().orc_direct_solve(dims, N, M, alpha, T, L, _dp(f), _dp(g), _dp(u), int(Mstop))
    return u


def modal_solve(dims, N, M, alpha, kx, s, ky=None, gq=None, T=1.0, L=1.0):
    """Time coefficients v[K, M] of the exact discrete solution for sine-mode
    forcing f = sum_q s[q](t_m) phi_q (Section 4.1 symbols at Dirichlet modes)."""
    kx = np.ascontiguousarray(kx, dtype=np.int32)
    K = kx.size
    ky = np.ascontiguousarray(ky if ky is not None else np.zeros(K), dtype=np.int32)
    s = _f64(s).reshape(K, M)
    gq = _f64(gq)
    v = np.zeros((K, M))
    _load().orc_modal_solve(dims, N, M, alpha, T, L, K, _ip(kx), _ip(ky), _dp(s), _dp(gq), _dp(v))
    return v


def modal_eval(dims, N, M, kx, v, pts, ky=None, L=1.0):
    """Evaluate the modal solution at sample points pts[:, (m, n, l)] (1-based)."""
    kx = np.ascontiguousarray(kx, dtype=np.int32)
    K = kx.size
    ky = np.ascontiguousarray(ky if ky is not None else np.zeros(K), dtype=np.int32)
    pts = np.ascontiguousarray(pts, dtype=np.int32).reshape(-1, 3)
    out = np.zeros(pts.shape[0])
    _load().orc_modal_eval(dims, N, M, L, K, _ip(kx), _ip(ky), _dp(_f64(v)), pts.shape[0],
                           _ip(pts), _dp(out))
    return out


def modal_grid(dims, N, M, kx, v, ky=None, L=1.0):
    """Full grid of the modal solution (small sizes only)."""
    if dims == 1:
        m, n = np.meshgrid(np.arange(1, M + 1), np.arange(1, N + 1), indexing="ij")
        pts = np.stack([m.ravel(), n.ravel(), np.ones(m.size, dtype=int)], axis=1)
        return modal_eval(dims, N, M, kx, v, pts, ky, L).reshape(M, N)
    m, l, n = np.meshgrid(np.arange(1, M + 1), np.arange(1, N + 1), np.arange(1, N + 1),
                          indexing="ij")
    pts = np.stack([m.ravel(), n.ravel(), l.ravel()], axis=1)
    return modal_eval(dims, N, M, kx, v, pts, ky, L).reshape(M, N, N)


def mittag_leffler(alpha, z):
    """E_alpha(z) by its defining series (Section 7), for |z| <= 1."""
    z = np.ascontiguousarray(np.asarray(z, dtype=np.float64))
    if np.abs(z).max(initial=0.0) > 1.0:
        raise ValueError("the series is summed for |z| <= 1 only")
    out = np.zeros_like(z)
    _load().orc_mittag_leffler(alpha, z.size, _dp(z), _dp(out))
    return out


def paper_test1_exact(N, M, alpha, T=1.0):
    """Exact solution E_alpha(-t^alpha) sin x of the first test problem of
    Section 7 (x in [0, pi], f = 0, g = sin x) on the grid, [M, N]."""
    t = T * np.arange(1, M + 1) / M
    x = np.pi * np.arange(1, N + 1) / (N + 1)
    return np.outer(mittag_leffler(alpha, -t ** alpha), np.sin(x))


def nl_solve(N, M, alpha, f, c=1.0, q=1.0, nu1=0, nu2=1, first=1, tol=1e-10, maxit=60, T=1.0):
    """Waveform relaxation FAS for the nonlinear problem of Section 7
    (D(u) = 1 + q u^2, convection c u_x, zero initial and boundary values);
    returns (u, hist)."""
    f = _f64(f)
    u = np.zeros((M, N))
    hist = np.zeros(maxit + 1)
    its = _load().orc_nl_solve(N, M, alpha, T, c, q, nu1, nu2, first, tol, maxit, _dp(f), _dp(u), _dp(hist))
    return u, hist[:its + 1]


def max_threads() -> int:
    """Threads the oracle's OpenMP loops use."""
    return int(_load().orc_max_threads())
