"""Host-side checks of the C ABI: the library loads, exports every symbol
include/mgwr.h declares, validates arguments before touching a device, and its
host-computed L1 weights agree with a high-precision evaluation (Section 2)."""
import ctypes
import os
import re

import numpy as np
import pytest

from paper_1608_05400_amd import binding

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_symbols():
    text = open(os.path.join(ROOT, "include", "mgwr.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(mgwr_[a-z0-9_]+)\s*\(", text)))


def test_library_exports_every_declared_symbol():
    lib = binding.load()
    names = declared_symbols()
    assert len(names) >= 19
    for n in names:
        assert hasattr(lib, n), n
    assert set(names) == set(binding.EXPORTED)


def test_default_options():
    o = binding.default_options()
    assert (o.nu1, o.nu2, o.gamma, o.maxit, o.norm, o.precision) == (1, 1, 1, 100, 0, 0)
    assert o.L == 1.0 and o.first_colour == 0
    assert (o.fft, o.inner_cycles, o.graph) == (1, 1, 1)


@pytest.mark.parametrize("M,alpha", [(64, 0.5), (16384, 0.3), (16384, 0.7), (8192, 0.1), (7, 0.9),
                                     (100, 1.0)])
def test_library_l1_weights_high_precision(M, alpha):
    import mpmath
    mpmath.mp.dps = 40
    c, r = binding.l1_weights(M, alpha)
    a = mpmath.mpf(alpha)
    cm = (mpmath.mpf(1) / M) ** (-a) / mpmath.gamma(2 - a)

    def dk(k):
        if k == 0:
            return mpmath.mpf(0)
        if k == 1:
            return mpmath.mpf(1)
        return mpmath.mpf(k) ** (1 - a) - mpmath.mpf(k - 1) ** (1 - a)

    assert abs(c - float(cm)) <= 2e-15 * float(cm)
    idx = sorted({1, 2, 3, 4, 5, 6, 9, 17, M // 2, M - 1, M} & set(range(1, M + 1)))
    for i in idx:
        ref = float(cm * (dk(i) - dk(i - 1)))
        if ref == 0.0:
            assert r[i - 1] == 0.0
        else:
            assert abs(r[i - 1] - ref) <= 2e-14 * abs(ref), (i, r[i - 1], ref)


def test_library_l1_weights_row_sums():
    import oracle
    M, alpha = 4096, 0.35
    c, r = binding.l1_weights(M, alpha)
    co, d, ro = oracle.l1_coeffs(M, alpha)
    assert np.allclose(np.cumsum(r), c * d[1:], rtol=1e-12)


@pytest.mark.parametrize("args", [(6, 16, 0.5, 1.0, 1), (7, 0, 0.5, 1.0, 1), (7, 16, 0.0, 1.0, 1),
                                  (7, 16, 1.2, 1.0, 1), (7, 16, 0.5, -1.0, 1), (7, 16, 0.5, 1.0, 3),
                                  (0, 16, 0.5, 1.0, 2)])
def test_create_rejects_bad_arguments_on_host(args):
    lib = binding.load()
    h = ctypes.c_void_p()
    rc = lib.mgwr_create(*args, ctypes.byref(h))
    assert rc == binding.MGWR_EINVAL
    assert not h.value
    assert binding.last_error()


def test_bad_options_rejected_on_host():
    lib = binding.load()
    h = ctypes.c_void_p()
    for kw in ({"nu1": 0, "nu2": 0}, {"gamma": 3}, {"precision": 9}, {"first_colour": 2},
               {"stall": 1.5}, {"L": -1.0}, {"inner_cycles": 0}, {"inner_cycles": 9}, {"fft": 3}):
        o = binding.default_options(**kw)
        rc = lib.mgwr_create_ex(7, 16, 0.5, 1.0, 1, ctypes.byref(o), ctypes.byref(h))
        assert rc == binding.MGWR_EINVAL, kw
