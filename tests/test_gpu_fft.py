"""GPU parity of the FFT route of the FP64 Toeplitz products (the causal
product as the leading block of a circulant product of length L >= 2M,
Section 5.1), through the C ABI, against the oracle.

Tolerances: an FFT convolution is accurate normwise, to a small multiple of
eps log2(L) times ||t||_1 max|x| per entry, so the products are compared
with 1e-12 of the term size sum_k |t_k| |x|; solves use the same bars as the
dense route (1e-10 FP64, 1e-8 mixed against the exact discrete solution).
"""
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


@pytest.mark.parametrize("M", [32, 33, 100, 1000, 4096])
@pytest.mark.parametrize("P", [1, 2, 7, 130])
def test_fft_product_matches_oracle_coefficients(B, M, P):
    alpha = 0.41
    rng = np.random.default_rng(M * 7 + P)
    X = rng.standard_normal((M, P))
    c, d, r = oracle.l1_coeffs(M, alpha)
    Tm = toeplitz_lower(r)
    ref = Tm @ X
    scale = (np.abs(Tm) @ np.abs(X)).max()
    with B.Solver(7, M, alpha, fft=2) as s:
        C = host(s.toeplitz_apply(dev(X), which=-1, precision="fp64"))
    assert relmax(C, ref, scale) <= 1e-12


@pytest.mark.parametrize("M,P", [(64, 31), (600, 200), (2048, 1023)])
def test_fft_inverse_column_product_is_line_solve(B, M, P):
    alpha = 0.6
    rng = np.random.default_rng(P)
    X = rng.standard_normal((M, P))
    c, d, r = oracle.l1_coeffs(M, alpha)
    with B.Solver(63, M, alpha, fft=2) as s:
        nl = s.levels()
        for lev in (0, nl // 2, nl - 1):
            n = 2 ** (lev + 1) - 1
            sigma = 2.0 * (n + 1) ** 2
            ref = linalg.solve_triangular(toeplitz_lower(r) + sigma * np.eye(M), X, lower=True)
            C = host(s.toeplitz_apply(dev(X), which=lev, precision="fp64"))
            assert relmax(C, ref) <= 1e-12, lev


@pytest.mark.parametrize("dims,N,M,alpha", [(1, 127, 200, 0.3), (2, 31, 64, 0.7), (1, 63, 33, 0.5)])
def test_fft_residual_and_sweep_match_oracle(B, dims, N, M, alpha):
    rng = np.random.default_rng(5)
    shape = (M, N) if dims == 1 else (M, N, N)
    f, u, g = rng.standard_normal(shape), rng.standard_normal(shape), rng.standard_normal(shape[1:])
    ref_r = oracle.residual(dims, N, M, alpha, f, u, g=g)
    ref_s = oracle.half_sweep(dims, N, M, alpha, 0, f, u, g=g)
    ref_s = oracle.half_sweep(dims, N, M, alpha, 1, f, ref_s, g=g)
    with B.Solver(N, M, alpha, dims=dims, fft=2) as s:
        R = host(s.residual(dev(f), dev(u), g=dev(g)))
        U = dev(u)
        s.smooth(dev(f), U, g=dev(g))
        U = host(U)
    scale = np.abs(f).max() + (2 * dims * (N + 1) ** 2 + 2 * oracle.l1_coeffs(M, alpha)[0]) * np.abs(u).max()
    assert relmax(R, ref_r, scale) <= 1e-12
    assert relmax(U, ref_s) <= 1e-12


@pytest.mark.parametrize("prec,tol", [("fp64", 1e-10), ("fp64r", 1e-10), ("fp32", 1e-8), ("bf16x3", 1e-8)])
def test_fft_solve_matches_direct_solve(B, prec, tol):
    w = W.random_modes_1d(255, 1500, 0.45, seed=77)
    f = w.forcing()
    ref = oracle.direct_solve(1, w.N, w.M, w.alpha, f)
    with B.Solver(w.N, w.M, w.alpha, precision=prec, fft=2) as s:
        U = torch.zeros(s.grid_shape, dtype=torch.float64, device="cuda")
        info = s.solve(dev(f), U, tol=1e-12)
        U = host(U)
    assert info["rc"] in (0, 2), info
    assert relmax(U, ref) <= tol, (info, relmax(U, ref))


@pytest.mark.parametrize("M", [40, 83, 255, 256, 300, 1100])
@pytest.mark.parametrize("first", [0, 1])
@pytest.mark.parametrize("prec", ["fp32", "bf16x3"])
def test_fft32_colour_panels_solve(B, M, first, prec):
    """1D mixed cycles on the FFT route: the first half-sweep writes its
    colour's points into a panel and the second merges it into U with its
    own (register passes below L = 512, radix-256 passes from 512 on; either
    colour first, so that each colour is the one with the extra point)."""
    N = 63
    f = np.random.default_rng(M + 7 * first).standard_normal((M, N))
    ref = oracle.direct_solve(1, N, M, 0.55, f)
    for nu in ((1, 1), (0, 1)):
        with B.Solver(N, M, 0.55, precision=prec, fft=2, first_colour=first, nu1=nu[0], nu2=nu[1],
                      maxit=200) as s:
            U = torch.zeros(s.grid_shape, dtype=torch.float64, device="cuda")
            info = s.solve(dev(f), U, tol=1e-12)
            U = host(U)
        assert info["rc"] in (0, 2), info
        assert relmax(U, ref) <= 1e-8, (nu, info, relmax(U, ref))


def test_fft_and_dense_routes_agree(B):
    """Same cycles, products by the two routes: the iterates agree to
    rounding and the iteration counts are the same."""
    w = W.random_modes_1d(511, 1024, 0.3, seed=78)
    f = w.forcing()
    outs = []
    for fft in (0, 2):
        with B.Solver(w.N, w.M, w.alpha, fft=fft) as s:
            U = torch.zeros(s.grid_shape, dtype=torch.float64, device="cuda")
            info = s.solve(dev(f), U, tol=1e-9)
            outs.append((host(U), info["iters"]))
    assert outs[0][1] == outs[1][1]
    assert relmax(outs[1][0], outs[0][0]) <= 1e-11


def test_fft_batch_with_uneven_problems(B):
    ws = [W.random_modes_1d(N, M, a, seed=90 + i) for i, (N, M, a) in
          enumerate([(63, 64, 0.5), (127, 1100, 0.2), (255, 40, 0.8), (31, 2048, 0.6)])]
    refs = [oracle.direct_solve(1, w.N, w.M, w.alpha, w.forcing()) for w in ws]
    b = B.Batch([w.N for w in ws], [w.M for w in ws], [w.alpha for w in ws], fft=2)
    us = [torch.zeros((w.M, w.N), dtype=torch.float64, device="cuda") for w in ws]
    rc, infos = b.solve([dev(w.forcing()) for w in ws], us, tol=1e-12)
    b.close()
    for u, ref, inf in zip(us, refs, infos):
        assert relmax(host(u), ref) <= 1e-10, inf


def test_fft_option_validated(B):
    with pytest.raises(B.MgwrError):
        B.Solver(15, 64, 0.5, fft=3)


@pytest.mark.parametrize("M", [64, 1000, 4096, 16384])
@pytest.mark.parametrize("P", [2, 129])
def test_fft32_product_matches_oracle_coefficients(B, M, P):
    """The FP32 FFT route (history products of the mixed cycles) on its own:
    FP32 arithmetic, so 1e-6 of the term size as for the dense FP32 kernel."""
    alpha = 0.7
    rng = np.random.default_rng(M + P)
    t = np.arange(1, M + 1) / M
    X = rng.standard_normal((M, P)) * t[:, None] ** 1.5
    c, d, r = oracle.l1_coeffs(M, alpha)
    Tm = toeplitz_lower(r)
    ref = Tm @ X
    scale = (np.abs(Tm) @ np.abs(X)).max()
    with B.Solver(7, M, alpha, fft=2) as s:
        C = host(s.toeplitz_apply(dev(X), which=-1, precision="fp32"))
    err = relmax(C, ref, scale)
    print(f"M {M} P {P}: max error / term size {err:.2e}")
    assert err <= 1e-6


# Transform lengths L = pow2 >= 2M from 512 to 65536: every first radix of
# the plans (2 ... 256) that the fused middle kernel (last forward pass,
# spectrum, first inverse pass) is built for, with one and two blocks of
# column pairs.
@pytest.mark.parametrize("M", [200, 300, 1000, 2048, 4096, 5000, 9000, 12345, 16384, 20000])
@pytest.mark.parametrize("P", [3, 33])
def test_fft_product_every_plan(B, M, P):
    alpha = 0.55
    rng = np.random.default_rng(3 * M + P)
    X = rng.standard_normal((M, P))
    c, d, r = oracle.l1_coeffs(M, alpha)
    # causal Toeplitz product = the first M terms of the full convolution
    ref = np.stack([np.convolve(r, X[:, p])[:M] for p in range(P)], axis=1)
    scale = np.stack([np.convolve(np.abs(r), np.abs(X[:, p]))[:M] for p in range(P)], axis=1).max()
    with B.Solver(7, M, alpha, fft=2) as s:
        C = host(s.toeplitz_apply(dev(X), which=-1, precision="fp64"))
        C32 = host(s.toeplitz_apply(dev(X), which=-1, precision="fp32"))
    assert relmax(C, ref, scale) <= 1e-12
    assert relmax(C32, ref, scale) <= 1e-6


# FP64 products with 512 < M <= 2048 take the kernel that keeps the whole
# transform on chip (one block per column pair): ragged column counts (a
# last pair of one column), M below the half transform length, and the
# scatter epilogue of the FP64 smoother on a level in natural order.
@pytest.mark.parametrize("M", [513, 1000, 1024, 1500, 2048])
@pytest.mark.parametrize("P", [1, 2, 9, 130])
def test_fft_product_on_chip(B, M, P):
    alpha = 0.45
    rng = np.random.default_rng(11 * M + P)
    X = rng.standard_normal((M, P))
    c, d, r = oracle.l1_coeffs(M, alpha)
    ref = np.stack([np.convolve(r, X[:, p])[:M] for p in range(P)], axis=1)
    scale = np.stack([np.convolve(np.abs(r), np.abs(X[:, p]))[:M] for p in range(P)], axis=1).max()
    with B.Solver(7, M, alpha, fft=2) as s:
        s.profile(True)
        C = host(s.toeplitz_apply(dev(X), which=-1, precision="fp64"))
        recs = s.profile_records()
        s.profile(False)
    assert relmax(C, ref, scale) <= 1e-12
    assert recs and all(rec["kernel"] >> 8 == 5 for rec in recs), [rec["name"] for rec in recs]


@pytest.mark.parametrize("N,M", [(31, 700), (15, 2048)])
def test_fft_on_chip_smoother_scatter(B, N, M):
    """One FP64 sweep on a 2D level in natural order (the scatter epilogue)
    with the on-chip products, against the oracle's sweep."""
    alpha = 0.5
    rng = np.random.default_rng(N + M)
    f = rng.standard_normal((M, N, N))
    u0 = rng.standard_normal((M, N, N))
    ref = oracle.half_sweep(2, N, M, alpha, 0, f, u0)
    ref = oracle.half_sweep(2, N, M, alpha, 1, f, ref)
    with B.Solver(N, M, alpha, dims=2, fft=2) as s:
        s.profile(True)
        U = dev(u0)
        s.smooth(dev(f), U)
        U = host(U)
        recs = s.profile_records()
        s.profile(False)
    assert any(rec["kernel"] == (5 << 8) | 1 for rec in recs), [rec["name"] for rec in recs]
    assert relmax(U, ref) <= 1e-10


@pytest.mark.parametrize("dims,N,M,alpha", [(1, 127, 200, 0.3), (2, 31, 64, 0.7), (1, 255, 600, 0.5), (2, 63, 520, 0.4)])
@pytest.mark.parametrize("first", [0, 1])
@pytest.mark.parametrize("nu", [(1, 1), (0, 1), (2, 1)])
@pytest.mark.parametrize("gamma", [1, 2])
def test_fft_cycle_matches_oracle(B, dims, N, M, alpha, first, nu, gamma):
    """One plain FP64 V- or W-cycle with every product on the FFT route, both
    colour orders and with and without pre-smoothing.  In a W-cycle the second
    visit of a coarse level starts from the first visit's result, not from
    zero (a regression case: its first half-sweep once took the right-hand
    side as if the level's iterate were zero)."""
    rng = np.random.default_rng(N + M + first)
    shape = (M, N) if dims == 1 else (M, N, N)
    f, u, g = rng.standard_normal(shape), rng.standard_normal(shape), rng.standard_normal(shape[1:])
    ref = oracle.vcycle(dims, N, M, alpha, f, u, g=g, nu1=nu[0], nu2=nu[1], gamma=gamma, first=first)
    with B.Solver(N, M, alpha, dims=dims, nu1=nu[0], nu2=nu[1], gamma=gamma, first_colour=first, fft=2) as s:
        U = dev(u)
        s.vcycle(dev(f), U, g=dev(g))
        U = host(U)
    assert relmax(U, ref) <= 1e-11


@pytest.mark.parametrize("prec,tol", [("fp64r", 1e-10), ("bf16x3", 1e-8)])
@pytest.mark.parametrize("first", [0, 1])
@pytest.mark.parametrize("dims,N,M,alpha", [(1, 255, 1500, 0.45), (2, 63, 600, 0.6)])
def test_fft_refinement_with_colour_residual(B, prec, tol, first, dims, N, M, alpha):
    """Refinement solves whose inner cycles compute the residual before
    restriction at the first colour only (FFT route, pre-smoothing): the
    outer FP64 residual brings them to the exact discrete solution."""
    if dims == 1:
        w = W.random_modes_1d(N, M, alpha, seed=80 + first)
    else:
        w = W.manufactured_2d(N, M, alpha)
    f = w.forcing()
    ref = oracle.direct_solve(dims, w.N, w.M, w.alpha, f)
    with B.Solver(w.N, w.M, w.alpha, dims=dims, precision=prec, first_colour=first, fft=2) as s:
        U = torch.zeros(s.grid_shape, dtype=torch.float64, device="cuda")
        info = s.solve(dev(f), U, tol=1e-12)
        U = host(U)
    assert info["rc"] in (0, 2), info
    assert relmax(U, ref) <= tol, (info, relmax(U, ref))


@pytest.mark.parametrize("cycles", [1, 2, 3])
def test_inner_cycles_per_refinement_step(B, cycles):
    """Refinement steps of 1, 2 or 3 cycles of the error equation reach the
    exact discrete solution; more cycles per step, fewer steps."""
    w = W.random_modes_1d(255, 1500, 0.6, seed=91)
    f = w.forcing()
    ref = oracle.direct_solve(1, w.N, w.M, w.alpha, f)
    with B.Solver(w.N, w.M, w.alpha, precision="bf16x3", inner_cycles=cycles) as s:
        U = torch.zeros(s.grid_shape, dtype=torch.float64, device="cuda")
        info = s.solve(dev(f), U, tol=1e-12)
        U = host(U)
    assert info["rc"] in (0, 2), info
    assert relmax(U, ref) <= 1e-8, (info, relmax(U, ref))
    print(f"inner_cycles {cycles}: {info['iters']} refinement steps")


@pytest.mark.parametrize("dims,N,M,alpha", [(1, 127, 700, 0.5), (2, 31, 520, 0.35)])
@pytest.mark.parametrize("cyc", [(1, 0, 2), (2, 1, 1), (1, 2, 2)])
def test_fft_refinement_cycle_shapes(B, dims, N, M, alpha, cyc):
    """Refinement with every product on the FFT route under other cycle shapes
    (nu1, nu2, gamma): W-cycles and several pre-smoothing sweeps, where the
    inner cycles restrict a one-colour residual."""
    nu1, nu2, gamma = cyc
    if dims == 1:
        w = W.random_modes_1d(N, M, alpha, seed=92)
    else:
        w = W.manufactured_2d(N, M, alpha)
    f = w.forcing()
    ref = oracle.direct_solve(dims, w.N, w.M, w.alpha, f)
    with B.Solver(w.N, w.M, w.alpha, dims=dims, precision="bf16x3", nu1=nu1, nu2=nu2, gamma=gamma, fft=2) as s:
        U = torch.zeros(s.grid_shape, dtype=torch.float64, device="cuda")
        info = s.solve(dev(f), U, tol=1e-12)
        U = host(U)
    assert info["rc"] in (0, 2), info
    assert relmax(U, ref) <= 1e-8, (info, relmax(U, ref))


@pytest.mark.parametrize("M", [40000, 70000])
@pytest.mark.parametrize("P", [2, 5])
def test_fft_product_long_time_lines(B, M, P):
    """Transform lengths beyond the benchmark's (L = 131072: a radix-2 first
    pass, the fused middle kernel with a radix-2 inverse stage); reference by
    a library FFT convolution of the oracle's coefficients, accurate normwise
    like the path itself."""
    from scipy import signal
    alpha = 0.35
    rng = np.random.default_rng(M + P)
    X = rng.standard_normal((M, P))
    c, d, r = oracle.l1_coeffs(M, alpha)
    ref = np.stack([signal.fftconvolve(r, X[:, p])[:M] for p in range(P)], axis=1)
    scale = np.abs(r).sum() * np.abs(X).max()
    with B.Solver(7, M, alpha, fft=2) as s:
        C = host(s.toeplitz_apply(dev(X), which=-1, precision="fp64"))
        C32 = host(s.toeplitz_apply(dev(X), which=-1, precision="fp32"))
    assert relmax(C, ref, scale) <= 1e-12
    assert relmax(C32, ref, scale) <= 1e-6


@pytest.mark.parametrize("prec,tol", [("fp64r", 1e-10), ("bf16x3", 1e-8)])
def test_fft_solve_long_time_line(B, prec, tol):
    """A solve at M = 40000 (transform length 131072) with three sine modes
    of forcing, against the oracle's modal solution (one forward substitution
    per mode)."""
    N, M, alpha = 63, 40000, 0.6
    t = np.arange(1, M + 1) / M
    kx = np.array([1, 4, 9], dtype=np.int32)
    s = np.stack([t ** 1.5, -0.5 * t ** 0.8, 0.25 * np.ones(M)])
    x = np.arange(1, N + 1) / (N + 1)
    f = s.T @ np.sin(np.pi * np.outer(kx, x))
    v = oracle.modal_solve(1, N, M, alpha, kx, s)
    ref = v.T @ np.sin(np.pi * np.outer(kx, x))
    with B.Solver(N, M, alpha, precision=prec, fft=2) as sv:
        U = torch.zeros((M, N), dtype=torch.float64, device="cuda")
        info = sv.solve(dev(f), U, tol=1e-12)
        U = host(U)
    assert info["rc"] in (0, 2), info
    assert relmax(U, ref) <= tol, (info, relmax(U, ref))
