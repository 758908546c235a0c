"""The oracle's C code under AddressSanitizer and UndefinedBehaviorSanitizer
(host only): a build of the same source with the sanitizers runs the oracle's
routines in a child process; any report fails the test.  CPU only."""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

SCRIPT = r"""
import math, numpy as np, oracle
rng = np.random.default_rng(0)
for dims, N, M in ((1, 31, 40), (2, 15, 12)):
    shape = (M, N) if dims == 1 else (M, N, N)
    f, u, g = rng.standard_normal(shape), rng.standard_normal(shape), rng.standard_normal(shape[1:])
    oracle.residual(dims, N, M, 0.4, f, u, g=g)
    for colour in (0, 1):
        oracle.half_sweep(dims, N, M, 0.4, colour, f, u, g=g)
    oracle.vcycle(dims, N, M, 0.4, f, u, g=g, nu1=1, nu2=1, gamma=2, first=1)
    oracle.mg_solve(dims, N, M, 0.4, f, g=g, tol=1e-8)
    oracle.direct_solve(dims, N, M, 0.4, f, g=g)
    kx = np.array([1, 3], dtype=np.int32)
    oracle.modal_grid(dims, N, M, kx, oracle.modal_solve(dims, N, M, 0.4, kx, np.ones((2, M)),
                                                         ky=kx if dims == 2 else None), ky=kx if dims == 2 else None)
oracle.l1_coeffs(100, 0.3)
oracle.mittag_leffler(0.6, -np.linspace(0, 1, 9))
oracle.nl_solve(15, 20, 0.5, np.ones((20, 15)))
print("ok")
"""


def test_oracle_under_address_and_ub_sanitizers(tmp_path):
    asan = subprocess.run(["gcc", "-print-file-name=libasan.so"], capture_output=True, text=True).stdout.strip()
    if not os.path.isabs(asan) or not os.path.exists(asan):
        pytest.skip("no libasan")
    lib = str(tmp_path / "liboracle_san.so")
    subprocess.run(["gcc", "-O1", "-g", "-fno-omit-frame-pointer", "-fsanitize=address,undefined",
                    "-fno-sanitize-recover=undefined", "-fPIC", "-shared", "-std=gnu11", "-o", lib,
                    os.path.join(ROOT, "oracle", "mgwr_oracle.c"), "-lm"], check=True)
    env = dict(os.environ, MGWR_ORACLE_LIB=lib, LD_PRELOAD=asan, ASAN_OPTIONS="detect_leaks=0",
               PYTHONPATH=ROOT, OMP_NUM_THREADS="1")
    res = subprocess.run([sys.executable, "-c", SCRIPT], capture_output=True, text=True, env=env, timeout=600)
    assert res.returncode == 0 and "ok" in res.stdout, res.stderr[-3000:]
    assert "runtime error" not in res.stderr and "AddressSanitizer" not in res.stderr, res.stderr[-3000:]
