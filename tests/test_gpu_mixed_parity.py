"""Element-wise parity of the mixed-precision cycle's own kernels.

In the refinement precisions the cycle on the error equation computes the
history part of every line solve and of every level's residual in FP32 or
split BF16 (the diagonal term, the stencils and every grid function stay
FP64).  ``mgwr_smooth`` and ``mgwr_vcycle`` run in the handle's precision,
so one smoothing step and one cycle are compared here point by point with
the oracle's FP64 half-sweep (Section 3, eq. red-black; Section 6, eq.
red-black_2d) and cycle (Algorithm 1).  The cycle's hierarchy is stored
split by colour, so covered are: the FFT route's epilogue writing the
diagonal term plus the history part into a colour's contiguous points (1D
and 2D), its one-colour and restricted residuals and the residual implied
by the sweep (cycles with pre-smoothing), the dense FP32 and split-BF16
epilogues adding the history part (``fft=0``), transform lengths below and
above 512 (register and LDS passes), both colour orders (in 1D the two
colours have an odd and an even number of points), ragged M.

Tolerances come from the unit roundoff u of the low precision and the
history share of the line solve.  With lambda the first column of
(T_M + sigma I)^{-1} and lambda_h the same without its first entry,
||lambda_h||_1 <= (c / sigma) lambda_0 (T_M + sigma I is an M-matrix whose
row sums are at least sigma), so the history part of a new value is at most
(c / sigma) of it.  A low-precision history product y = Lambda_h b obeys
  |y_hat - y| <= kappa u ||lambda_h||_1 max|b|,
with kappa = M + 3 for the dense products (operands rounded once, at most M
terms accumulated in FP32; split BF16 adds 3 2^-16 per term for the
representation of each operand by hi + lo and the dropped lo*lo term) and
kappa = 12 log2(L) sqrt(2M) for the FFT route (the normwise error of a
length-L transform pair and the spectrum product, 2 log2(L) radix-2 stages
of at most 6u each, bounded in the max norm by the 2-norm of a complex
column pair of length M).  An index error (a wrong neighbour, colour point
or partner write) moves a value by a sizeable fraction of max|x|, orders of
magnitude above these bounds on every case here.
"""
import math

import numpy as np
import pytest
from scipy import linalg

import oracle
from paper_1608_05400_amd import workloads as W

torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu

U_FP32 = 2.0 ** -24
U_SPLIT = 3 * 2.0 ** -16   # per term of a split-BF16 product (hi*hi + hi*lo + lo*hi)


@pytest.fixture(scope="module")
def B():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1608_05400_amd import binding
    binding.load()
    return binding


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64)).cuda()


def host(t):
    torch.cuda.synchronize()
    return t.cpu().numpy()


def fft_len(M):
    L = 64
    while L < 2 * M:
        L *= 2
    return L


def hist_norm(M, alpha, sigma):
    """||lambda_h||_1 of the inverse column of T_M + sigma I, from the oracle's
    L1 weights and a triangular solve (a library primitive)."""
    c, d, r = oracle.l1_coeffs(M, alpha)
    T = linalg.toeplitz(r, np.zeros_like(r))
    e = np.zeros(M)
    e[0] = 1.0
    lam = linalg.solve_triangular(T + sigma * np.eye(M), e, lower=True)
    return float(np.abs(lam[1:]).sum()), c


def kappa_u(prec, route, M):
    """kappa u of the history products (see the module docstring)."""
    if route == "fft":
        return 12.0 * math.log2(fft_len(M)) * math.sqrt(2.0 * M) * U_FP32
    per_term = U_SPLIT if prec == "bf16x3" else 2 * U_FP32
    return per_term + (M + 1) * U_FP32


def sigma_of(dims, n, L=1.0):
    return 2.0 * dims * ((n + 1) / L) ** 2


# ---------------------------------------------------------------------------
# one smoothing step (both half-sweeps) of the finest level

SWEEP_CASES = [
    (1, 255, 100, 0.5),    # L = 256: register passes; colour 0 has 127 points (< 128: FP32 dense)
    (1, 511, 300, 0.3),    # L = 1024: LDS passes; 255 / 256 points
    (1, 1023, 2000, 0.7),  # L = 4096
    (1, 15, 300, 0.9),     # c > 0.1 sigma: FFT route in FP64 there
    (2, 31, 200, 0.4),     # 2D: colour scatter of the diagonal term
    (2, 63, 257, 0.6),     # ragged M
]


@pytest.mark.parametrize("route", ["fft", "dense"])
@pytest.mark.parametrize("prec", ["fp32", "bf16x3"])
@pytest.mark.parametrize("first", [0, 1])
@pytest.mark.parametrize("dims,N,M,alpha", SWEEP_CASES)
def test_mixed_sweep_matches_oracle(B, dims, N, M, alpha, first, prec, route):
    rng = np.random.default_rng(N * 7 + M + first)
    shape = (M, N) if dims == 1 else (M, N, N)
    f, u, g = rng.standard_normal(shape), rng.standard_normal(shape), rng.standard_normal(shape[1:])
    mid = oracle.half_sweep(dims, N, M, alpha, first, f, u, g=g)
    ref = oracle.half_sweep(dims, N, M, alpha, 1 - first, f, mid, g=g)
    fft = 2 if route == "fft" else 0
    with B.Solver(N, M, alpha, dims=dims, first_colour=first, precision=prec, fft=fft) as s:
        U = dev(u)
        s.smooth(dev(f), U, g=dev(g), sweeps=1)
        U = host(U)
    sigma = sigma_of(dims, N)
    hn, c = hist_norm(M, alpha, sigma)
    ih2 = (N + 1) ** 2
    # right-hand sides of the two half-sweeps: |f| + c |g| (c d_m <= c) + the
    # neighbours (2 dims of them) / h^2
    bmax = [np.abs(f).max() + c * np.abs(g).max() + 2 * dims * ih2 * np.abs(x).max() for x in (u, mid)]
    # the first half-sweep's error enters the second's right-hand sides times
    # (neighbours / h^2) lambda_0 <= 1 (sigma = 2 dims / h^2)
    ku = kappa_u(prec, route, M)
    tol = ku * hn * (2 * bmax[0] + bmax[1]) + 1e-12 * np.abs(ref).max()
    err = np.abs(U - ref).max()
    print(f"{dims}D N {N} M {M} first {first} {prec} {route}: err {err:.3e} tol {tol:.3e} "
          f"(c/sigma {c / sigma:.2e}, err/max|x| {err / np.abs(ref).max():.2e})")
    assert err <= tol
    # and far below what an index error would give
    assert tol <= 1e-3 * np.abs(ref).max()


# ---------------------------------------------------------------------------
# one cycle of the error equation (u = 0 on entry), as in the refinement

CYCLE_CASES = [
    (1, 255, 300, 0.5, 1, 1, 1),
    (1, 1023, 1024, 0.7, 1, 1, 1),
    (1, 511, 600, 0.3, 1, 0, 2),      # W(1,0)
    (1, 127, 3000, 0.6, 0, 1, 1),     # V(0,1): the full residual before restriction
    (2, 31, 200, 0.4, 1, 1, 1),
    (2, 63, 129, 0.6, 1, 1, 1),
]


@pytest.mark.parametrize("route", ["fft", "dense"])
@pytest.mark.parametrize("prec", ["fp32", "bf16x3"])
@pytest.mark.parametrize("first", [0, 1])
@pytest.mark.parametrize("dims,N,M,alpha,nu1,nu2,gamma", CYCLE_CASES)
def test_mixed_cycle_matches_oracle(B, dims, N, M, alpha, nu1, nu2, gamma, first, prec, route):
    """Pre-smoothing makes the residual before restriction the first
    colour's only (epilogue 8; in 1D with colour 0 first it is written
    restricted, epilogue 9); the coarse levels' products take FP32 or split
    BF16 by their width, the FFT route in FP32 where c <= 0.1 sigma."""
    rng = np.random.default_rng(N + 3 * M + first)
    shape = (M, N) if dims == 1 else (M, N, N)
    f = rng.standard_normal(shape)
    u0 = np.zeros(shape)
    ref = oracle.vcycle(dims, N, M, alpha, f, u0, nu1=nu1, nu2=nu2, gamma=gamma, first=first)
    fft = 2 if route == "fft" else 0
    with B.Solver(N, M, alpha, dims=dims, first_colour=first, precision=prec, fft=fft, nu1=nu1, nu2=nu2,
                  gamma=gamma) as s:
        U = dev(u0)
        s.vcycle(dev(f), U)
        U = host(U)
    # error budget: every level's low-precision history products, relative
    # to the correction, with the share c / sigma_l capped at 1 (the coarse
    # levels, where the history carries the whole line solve), times 8 for
    # the transfers and the coarse-grid correction between levels
    ku = kappa_u(prec, route, M)
    c = oracle.l1_coeffs(M, alpha)[0]
    share = 0.0
    n = N
    while True:
        share += min(1.0, c / sigma_of(dims, n))
        if n == 1:
            break
        n = (n - 1) // 2
    scale = np.abs(ref).max()
    tol = 8.0 * gamma * ku * share * scale + 1e-11 * scale
    err = np.abs(U - ref).max()
    print(f"{dims}D N {N} M {M} V({nu1},{nu2}) gamma {gamma} first {first} {prec} {route}: "
          f"err/max|u| {err / scale:.3e} tol/max|u| {tol / scale:.3e}")
    assert err <= tol
    assert tol <= 2e-2 * scale


# ---------------------------------------------------------------------------
# iteration counts: the low-precision cycles contract like the FP64 one

def _iters(B, w, prec):
    f = w.forcing_torch("cuda").contiguous()
    with B.Solver(w.N, w.M, w.alpha, dims=w.dims, precision=prec) as s:
        U = torch.zeros(s.grid_shape, dtype=torch.float64, device="cuda")
        info = s.solve(f, U, tol=1e-10)
    assert info["status"] == "ok", (prec, info)
    return info["iters"]


@pytest.mark.parametrize("wl", ["config2_0.3", "config2_0.7", "1d_1023_4096"])
def test_mixed_iterations_bounded_by_fp64_refinement(B, wl):
    """A defect in a low-precision kernel that only slowed the cycle would be
    hidden by the FP64 refinement; so the FP32 and split-BF16 refinements
    must take at most one refinement step more than the FP64 one."""
    if wl.startswith("config2"):
        w = W.config2(float(wl.split("_")[1]))
    else:
        w = W.random_modes_1d(1023, 4096, 0.5, seed=91)
    n64 = _iters(B, w, "fp64r")
    for prec in ("fp32", "bf16x3"):
        n = _iters(B, w, prec)
        print(f"{wl}: {prec} {n} refinement steps, fp64r {n64}")
        assert n <= n64 + 1, (prec, n, n64)
