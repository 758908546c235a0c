"""GPU parity: the HIP path (through the C ABI) against the CPU oracle.

Every reference value here comes from ``oracle`` (or from a library primitive
applied to oracle coefficients); no expected value comes from the HIP path.
Tolerances (relative, max norm):
  * Toeplitz products, residual, one sweep, one cycle in FP64: the two sides
    compute the same sums in a different order, so they agree to a small
    multiple of the unit roundoff times the size of the terms (1e-12);
  * FP64 solves: 1e-10 against the exact discrete solution;
  * FP32 / split-BF16 products: 1e-6 / 5e-5 of the term size (24- / ~16-bit
    operands, FP32 accumulation);
  * mixed-precision solves: 1e-8 against the exact discrete solution.
"""
import math

import numpy as np
import pytest
from scipy import linalg

import oracle
from paper_1608_05400_amd import workloads as W

torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu


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


def relmax(a, b, scale=None):
    s = np.abs(b).max() if scale is None else scale
    return np.abs(a - b).max() / (s if s > 0 else 1.0)


def toeplitz_lower(col):
    return linalg.toeplitz(col, np.zeros_like(col))


# ---------------------------------------------------------------------------
# Toeplitz products (history GEMMs)

@pytest.mark.parametrize("M", [1, 37, 128, 300])
@pytest.mark.parametrize("P", [1, 5, 33, 64, 130])
def test_toeplitz_product_fp64(B, M, P):
    alpha = 0.37
    rng = np.random.default_rng(M * 1000 + P)
    X = rng.standard_normal((M, P))
    c, d, r = oracle.l1_coeffs(M, alpha)
    ref = toeplitz_lower(r) @ X
    scale = (np.abs(toeplitz_lower(r)) @ np.abs(X)).max()
    with B.Solver(7, M, alpha, dims=1) as s:
        C = host(s.toeplitz_apply(dev(X), which=-1, precision="fp64"))
    assert relmax(C, ref, scale) <= 1e-13


@pytest.mark.parametrize("M,P", [(64, 31), (257, 200), (512, 1023)])
def test_inverse_toeplitz_product_is_line_solve(B, M, P):
    """Smoother kernel: the product with the precomputed inverse column solves
    (T_M + sigma I) x = b exactly (Section 5.2) on every level."""
    alpha = 0.6
    rng = np.random.default_rng(P)
    X = rng.standard_normal((M, P))
    c, d, r = oracle.l1_coeffs(M, alpha)
    N = 63
    with B.Solver(N, M, alpha, dims=1) as s:
        nl = s.levels()
        for lev in (0, nl // 2, nl - 1):
            n = 2 ** (lev + 1) - 1
            sigma = 2.0 * (n + 1) ** 2
            ref = linalg.solve_triangular(toeplitz_lower(r) + sigma * np.eye(M), X, lower=True)
            C = host(s.toeplitz_apply(dev(X), which=lev, precision="fp64"))
            assert relmax(C, ref) <= 1e-12, lev


@pytest.mark.parametrize("prec,tol", [("fp32", 1e-6), ("bf16x3", 5e-5)])
@pytest.mark.parametrize("M,P", [(100, 40), (384, 300), (1024, 129)])
def test_toeplitz_product_low_precision(B, prec, tol, M, P):
    alpha = 0.45
    rng = np.random.default_rng(M + P)
    X = rng.standard_normal((M, P))
    c, d, r = oracle.l1_coeffs(M, alpha)
    Tm = toeplitz_lower(r)
    ref = Tm @ X
    scale = (np.abs(Tm) @ np.abs(X)).max()
    with B.Solver(7, M, alpha, dims=1, precision=prec) as s:
        C = host(s.toeplitz_apply(dev(X), which=-1, precision=prec))
    assert relmax(C, ref, scale) <= tol


# ---------------------------------------------------------------------------
# residual, sweep, cycle against the oracle's step references

CASES = [(1, 63, 64, 0.5), (1, 127, 37, 0.3), (1, 255, 200, 0.8), (2, 15, 24, 0.4), (2, 31, 40, 0.7)]


def _rand_problem(dims, N, M, seed):
    rng = np.random.default_rng(seed)
    shape = (M, N) if dims == 1 else (M, N, N)
    return rng.standard_normal(shape), rng.standard_normal(shape), rng.standard_normal(shape[1:])


@pytest.mark.parametrize("dims,N,M,alpha", CASES)
def test_residual_matches_oracle(B, dims, N, M, alpha):
    f, u, g = _rand_problem(dims, N, M, 1)
    ref = oracle.residual(dims, N, M, alpha, f, u, g=g)
    with B.Solver(N, M, alpha, dims=dims) as s:
        R, nrm = s.residual(dev(f), dev(u), g=dev(g), norms=True)
        R = host(R)
    scale = np.abs(f).max() + (2 * dims * (N + 1) ** 2 + 2 * oracle.l1_coeffs(M, alpha)[0]) * np.abs(u).max()
    assert relmax(R, ref, scale) <= 1e-13
    assert nrm[0] == pytest.approx(np.abs(ref).max(), rel=1e-10)
    assert nrm[1] == pytest.approx(np.linalg.norm(ref), rel=1e-10)


@pytest.mark.parametrize("dims,N,M,alpha", CASES)
@pytest.mark.parametrize("first", [0, 1])
def test_one_sweep_matches_oracle(B, dims, N, M, alpha, first):
    f, u, g = _rand_problem(dims, N, M, 2)
    ref = oracle.half_sweep(dims, N, M, alpha, first, f, u, g=g)
    ref = oracle.half_sweep(dims, N, M, alpha, 1 - first, f, ref, g=g)
    with B.Solver(N, M, alpha, dims=dims, first_colour=first) as s:
        U = dev(u)
        s.smooth(dev(f), U, g=dev(g), sweeps=1)
        U = host(U)
    assert relmax(U, ref) <= 1e-12


@pytest.mark.parametrize("dims,N,M,alpha", CASES)
@pytest.mark.parametrize("nu", [(1, 1), (0, 1)])
def test_one_cycle_matches_oracle(B, dims, N, M, alpha, nu):
    f, u, g = _rand_problem(dims, N, M, 3)
    ref = oracle.vcycle(dims, N, M, alpha, f, u, g=g, nu1=nu[0], nu2=nu[1])
    with B.Solver(N, M, alpha, dims=dims, nu1=nu[0], nu2=nu[1]) as s:
        U = dev(u)
        s.vcycle(dev(f), U, g=dev(g))
        U = host(U)
    assert relmax(U, ref) <= 1e-11


def test_w_cycle_matches_oracle(B):
    dims, N, M, alpha = 1, 63, 48, 0.4
    f, u, g = _rand_problem(dims, N, M, 4)
    ref = oracle.vcycle(dims, N, M, alpha, f, u, g=g, nu1=1, nu2=0, gamma=2)
    with B.Solver(N, M, alpha, dims=dims, nu1=1, nu2=0, gamma=2) as s:
        U = dev(u)
        s.vcycle(dev(f), U, g=dev(g))
        U = host(U)
    assert relmax(U, ref) <= 1e-11


# ---------------------------------------------------------------------------
# solves against the exact discrete solution

@pytest.mark.parametrize("prec,tol", [("fp64", 1e-10), ("fp64r", 1e-10), ("fp32", 1e-8), ("bf16x3", 1e-8)])
def test_config1_solve(B, prec, tol):
    """1D, N = 63, M = 64, alpha = 0.5, u = t^2 sin(pi x) manufactured forcing."""
    w = W.manufactured_1d()
    f = w.forcing()
    ref = oracle.direct_solve(1, w.N, w.M, w.alpha, f)
    with B.Solver(w.N, w.M, w.alpha, dims=1, precision=prec) as s:
        U = torch.zeros(s.grid_shape, dtype=torch.float64, device="cuda")
        info = s.solve(dev(f), U, tol=1e-13)
        U = host(U)
    assert info["rc"] in (0, 2), info
    assert relmax(U, ref) <= tol, (info, relmax(U, ref))


@pytest.mark.parametrize("prec,tol", [("fp64", 1e-10), ("fp32", 1e-8), ("bf16x3", 1e-8)])
@pytest.mark.parametrize("dims,N,M,alpha", [(1, 511, 1024, 0.3), (2, 63, 256, 0.4)])
def test_solve_with_initial_condition(B, prec, tol, dims, N, M, alpha):
    rng = np.random.default_rng(7)
    K = 5
    kx = rng.integers(1, 9, size=K)
    ky = rng.integers(1, 9, size=K) if dims == 2 else np.zeros(K, int)
    t = np.arange(1, M + 1) / M
    s_ = rng.standard_normal((K, 1)) * t[None, :] ** 1.5
    w = W.Workload(dims, N, M, alpha, 1.0, 1.0, kx.astype(np.int32), ky.astype(np.int32), s_)
    f = w.forcing()
    x = np.arange(1, N + 1) / (N + 1)
    g = np.sin(np.pi * x) if dims == 1 else np.outer(np.sin(np.pi * x), np.sin(2 * np.pi * x))
    ref = oracle.direct_solve(dims, N, M, alpha, f, g=g)
    with B.Solver(N, M, alpha, dims=dims, precision=prec) as s:
        U = torch.zeros(s.grid_shape, dtype=torch.float64, device="cuda")
        info = s.solve(dev(f), U, g=dev(g), tol=1e-12)
        U = host(U)
    assert info["rc"] in (0, 2), info
    assert relmax(U, ref) <= tol, (info, relmax(U, ref))


def test_solve_iteration_counts_follow_oracle(B):
    """The GPU FP64 iteration is Algorithm 1: same residual history as the
    oracle's iteration up to rounding."""
    dims, N, M, alpha = 1, 127, 128, 0.4
    w = W.paper_test1(N, M, alpha)
    g = W.paper_test1_g(w)
    f = np.zeros((M, N))
    _, hist = oracle.mg_solve(1, N, M, alpha, f, g=g, nu1=0, nu2=1, first=1, norm=1, tol=1e-10, L=math.pi)
    with B.Solver(N, M, alpha, dims=1, nu1=0, nu2=1, first_colour=1, norm="l2", L=math.pi) as s:
        U = torch.zeros(s.grid_shape, dtype=torch.float64, device="cuda")
        info = s.solve(dev(f), U, g=dev(g), tol=1e-10)
    assert info["iters"] == len(hist) - 1
    gh = np.array(info["hist"])
    big = hist >= 1e-8 * hist[0]
    # above the rounding floor the histories agree closely; near it (about
    # 1e-11 of r0 here) they differ by rounding noise of the two residuals
    np.testing.assert_allclose(gh[big], hist[big], rtol=1e-4)
    np.testing.assert_allclose(gh[~big], hist[~big], rtol=3e-2)


# ---------------------------------------------------------------------------
# edge cases

def test_single_point_grid_is_direct_solve(B):
    N, M, alpha = 1, 50, 0.5
    rng = np.random.default_rng(9)
    f = rng.standard_normal((M, N))
    ref = oracle.direct_solve(1, N, M, alpha, f)
    with B.Solver(N, M, alpha) as s:
        U = torch.zeros((M, N), dtype=torch.float64, device="cuda")
        info = s.solve(dev(f), U, tol=1e-14)
        U = host(U)
    assert info["iters"] <= 1
    assert relmax(U, ref) <= 1e-13


def test_single_time_step(B):
    N, M, alpha = 31, 1, 0.5
    rng = np.random.default_rng(10)
    f = rng.standard_normal((M, N))
    ref = oracle.direct_solve(1, N, M, alpha, f)
    with B.Solver(N, M, alpha) as s:
        U = torch.zeros((M, N), dtype=torch.float64, device="cuda")
        s.solve(dev(f), U, tol=1e-13)
        U = host(U)
    assert relmax(U, ref) <= 1e-10


def test_nonfinite_input_is_reported(B):
    N, M = 15, 16
    f = np.zeros((M, N))
    f[3, 4] = np.nan
    with B.Solver(N, M, 0.5) as s:
        U = torch.zeros((M, N), dtype=torch.float64, device="cuda")
        info = s.solve(dev(f), U, tol=1e-10, raise_on_error=False)
    assert info["rc"] == B.MGWR_ENONFINITE


def test_bad_arguments_rejected(B):
    with pytest.raises(B.MgwrError):
        B.Solver(6, 16, 0.5)
    with pytest.raises(B.MgwrError):
        B.Solver(7, 16, 1.5)
    with B.Solver(7, 16, 0.5) as s:
        bad = torch.zeros((16, 8), dtype=torch.float64, device="cuda")
        with pytest.raises(ValueError):
            s.vcycle(bad, bad)


def test_runs_are_bitwise_deterministic(B):
    dims, N, M, alpha = 1, 255, 300, 0.6
    f, _, g = _rand_problem(dims, N, M, 11)
    outs = []
    for _ in range(2):
        with B.Solver(N, M, alpha) as s:
            U = torch.zeros((M, N), dtype=torch.float64, device="cuda")
            s.solve(dev(f), U, g=dev(g), tol=1e-12)
            outs.append(host(U))
    assert np.array_equal(outs[0], outs[1])


# ---------------------------------------------------------------------------
# full workload sizes, in the launch configuration the benchmark times:
# sampled outputs against the exact discrete solution from the oracle's modal
# solve (every workload forcing is a finite sum of sine modes)

def _sampled_modal_error(w, U, npts=3000, seed=5):
    rng = np.random.default_rng(seed)
    v = oracle.modal_solve(w.dims, w.N, w.M, w.alpha, w.kx, w.s, ky=w.ky)
    m = rng.integers(1, w.M + 1, size=npts)
    m[:50] = w.M
    m[50:100] = 1
    n = rng.integers(1, w.N + 1, size=npts)
    l = rng.integers(1, w.N + 1, size=npts) if w.dims == 2 else np.ones(npts, dtype=np.int64)
    ref = oracle.modal_eval(w.dims, w.N, w.M, w.kx, v, np.stack([m, n, l], 1), ky=w.ky)
    if w.dims == 1:
        idx = (m - 1) * w.N + (n - 1)
    else:
        idx = (m - 1) * w.N * w.N + (l - 1) * w.N + (n - 1)
    got = U.reshape(-1)[torch.from_numpy(idx).cuda()].cpu().numpy()
    return np.abs(got - ref).max() / np.abs(ref).max()


@pytest.mark.parametrize("prec,tol", [("bf16x3", 1e-8), ("fp64r", 1e-10), ("fp32", 1e-8)])
@pytest.mark.parametrize("alpha", [0.3, 0.7])
def test_config2_full_size(B, prec, tol, alpha):
    """1D, N = 4095, M = 16384: reaches a 1e-10 relative FP64 residual."""
    w = W.config2(alpha)
    f = w.forcing_torch("cuda").contiguous()
    with B.Solver(w.N, w.M, w.alpha, precision=prec) as s:
        U = torch.zeros(s.grid_shape, dtype=torch.float64, device="cuda")
        info = s.solve(f, U, tol=1e-10)
        torch.cuda.synchronize()
        err = _sampled_modal_error(w, U)
    assert info["status"] == "ok" and info["relres"] <= 1e-10, info
    assert err <= tol, err


def test_config2_plain_fp64_reaches_its_floor(B):
    """Plain FP64 stops at the rounding floor of the residual for h = 1/4096
    (about 2e-9 relative in the max norm) with the solution accurate."""
    w = W.config2(0.3)
    f = w.forcing_torch("cuda").contiguous()
    with B.Solver(w.N, w.M, w.alpha, precision="fp64") as s:
        U = torch.zeros(s.grid_shape, dtype=torch.float64, device="cuda")
        info = s.solve(f, U, tol=1e-10)
        torch.cuda.synchronize()
        err = _sampled_modal_error(w, U)
    assert info["status"] in ("ok", "stagnated") and info["relres"] <= 1e-8, info
    assert err <= 1e-10, err


@pytest.mark.parametrize("prec,tol", [("bf16x3", 1e-8), ("fp32", 1e-8), ("fp64", 1e-10)])
def test_config3_2d_full_size(B, prec, tol):
    """2D, N = 511, M = 2048, alpha = 0.4, u = t^2 sin(pi x) sin(pi y): every
    precision reaches the 1e-10 relative FP64 residual of the benchmark."""
    w = W.manufactured_2d(511, 2048, 0.4)
    f = w.forcing_torch("cuda").contiguous()
    with B.Solver(w.N, w.M, w.alpha, dims=2, precision=prec) as s:
        U = torch.zeros(s.grid_shape, dtype=torch.float64, device="cuda")
        info = s.solve(f, U, tol=1e-10)
        torch.cuda.synchronize()
        err = _sampled_modal_error(w, U)
    print(prec, info["iters"], info["relres"], info["hist"], err)
    assert info["status"] == "ok" and info["relres"] <= 1e-10, info
    assert err <= tol, err


def test_config5_2d_nonsmooth_full_size(B):
    """2D, N = 1023, M = 1024, alpha = 0.3, u = (t^a + t^2) sin sin, split-BF16."""
    w = W.nonsmooth_2d(1023, 1024, 0.3)
    f = w.forcing_torch("cuda").contiguous()
    with B.Solver(w.N, w.M, w.alpha, dims=2, precision="bf16x3") as s:
        U = torch.zeros(s.grid_shape, dtype=torch.float64, device="cuda")
        info = s.solve(f, U, tol=1e-10)
        torch.cuda.synchronize()
        err = _sampled_modal_error(w, U)
    assert info["status"] == "ok" and info["relres"] <= 1e-10, info
    assert err <= 1e-8, err
