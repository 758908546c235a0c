"""Seeded random combinations of the solver's options through the C ABI,
against the oracle: one plain FP64 cycle (V or W, any pre/post-smoothing,
either colour first, dense or FFT products, inverse-column or D&C smoother,
1D or 2D, ragged M) must equal the oracle's cycle, and a solve in a mixed
precision must reach the exact discrete solution.  Faults of rarely combined
options (one was a W-cycle fault of the FFT route) show up here.
"""
import numpy as np
import pytest

import oracle

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


def draw(seed):
    rng = np.random.default_rng(1000 + seed)
    dims = int(rng.integers(1, 3))
    N = int(rng.choice([7, 15, 31, 63] if dims == 1 else [7, 15, 31]))
    M = int(rng.integers(1, 700 if dims == 1 else 300))
    alpha = float(rng.uniform(0.05, 1.0))
    nu1, nu2 = [int(v) for v in rng.integers(0, 3, size=2)]
    if nu1 + nu2 == 0:
        nu2 = 1
    gamma = int(rng.integers(1, 3))
    first = int(rng.integers(0, 2))
    fft = int(rng.choice([0, 2])) if M >= 32 else 0
    smoother = str(rng.choice(["inverse", "dc"]))
    dc_block = int(rng.choice([128, 256])) if smoother == "dc" else 0
    prec = str(rng.choice(["fp32", "bf16x3", "fp64r"]))
    return dict(dims=dims, N=N, M=M, alpha=alpha, nu1=nu1, nu2=nu2, gamma=gamma, first=first, fft=fft,
                smoother=smoother, dc_block=dc_block, prec=prec, rng=rng)


@pytest.mark.parametrize("seed", range(120))
def test_random_fp64_cycle_matches_oracle(B, seed):
    c = draw(seed)
    dims, N, M, alpha, rng = c["dims"], c["N"], c["M"], c["alpha"], c["rng"]
    shape = (M, N) if dims == 1 else (M, N, N)
    f, u, g = rng.standard_normal(shape), rng.standard_normal(shape), rng.standard_normal(shape[1:])
    print({k: v for k, v in c.items() if k != "rng"}, flush=True)
    ref = oracle.vcycle(dims, N, M, alpha, f, u, g=g, nu1=c["nu1"], nu2=c["nu2"], gamma=c["gamma"],
                        first=c["first"])
    with B.Solver(N, M, alpha, dims=dims, nu1=c["nu1"], nu2=c["nu2"], gamma=c["gamma"], first_colour=c["first"],
                  fft=c["fft"], smoother=c["smoother"], dc_block=c["dc_block"]) as s:
        U = dev(u)
        s.vcycle(dev(f), U, g=dev(g))
        U = host(U)
    assert np.abs(U - ref).max() <= 1e-11 * np.abs(ref).max()


@pytest.mark.parametrize("seed", range(50))
def test_random_mixed_solve_reaches_direct_solution(B, seed):
    c = draw(seed)
    dims, N, M, alpha, rng = c["dims"], c["N"], max(c["M"], 2), c["alpha"], c["rng"]
    shape = (M, N) if dims == 1 else (M, N, N)
    f = rng.standard_normal(shape)
    print({k: v for k, v in c.items() if k != "rng"}, flush=True)
    ref = oracle.direct_solve(dims, N, M, alpha, f)
    with B.Solver(N, M, alpha, dims=dims, nu1=c["nu1"], nu2=c["nu2"], gamma=c["gamma"], first_colour=c["first"],
                  fft=c["fft"], smoother=c["smoother"], dc_block=c["dc_block"], precision=c["prec"],
                  maxit=200) as s:
        U = torch.zeros(shape, dtype=torch.float64, device="cuda")
        info = s.solve(dev(f), U, tol=1e-12)
        U = host(U)
    assert info["rc"] in (0, 2), info
    assert np.abs(U - ref).max() <= 1e-8 * np.abs(ref).max(), info


@pytest.mark.parametrize("seed", range(15))
def test_random_batch_solve_reaches_direct_solutions(B, seed):
    """A batch of uneven problems under one drawn set of options."""
    c = draw(200 + seed)
    rng = c["rng"]
    dims = c["dims"]
    count = int(rng.integers(2, 7))
    Ns = [int(rng.choice([7, 15, 31, 63] if dims == 1 else [7, 15])) for _ in range(count)]
    Ms = [int(rng.integers(2, 400 if dims == 1 else 150)) for _ in range(count)]
    als = [float(rng.uniform(0.05, 1.0)) for _ in range(count)]
    fs = [rng.standard_normal((M, N) if dims == 1 else (M, N, N)) for N, M in zip(Ns, Ms)]
    print({k: v for k, v in c.items() if k != "rng"}, Ns, Ms, flush=True)
    refs = [oracle.direct_solve(dims, N, M, a, f) for N, M, a, f in zip(Ns, Ms, als, fs)]
    b = B.Batch(Ns, Ms, als, dims=dims, nu1=c["nu1"], nu2=c["nu2"], gamma=c["gamma"], first_colour=c["first"],
                fft=c["fft"], smoother=c["smoother"], dc_block=c["dc_block"], precision=c["prec"], maxit=200)
    us = [torch.zeros(f.shape, dtype=torch.float64, device="cuda") for f in fs]
    rc, infos = b.solve([dev(f) for f in fs], us, tol=1e-12)
    b.close()
    for u, ref, inf in zip(us, refs, infos):
        assert np.abs(host(u) - ref).max() <= 1e-8 * np.abs(ref).max(), inf


@pytest.mark.parametrize("seed", range(30))
def test_random_fas_cycles_match_oracle(B, seed):
    """The nonlinear FAS solver under drawn sizes, coefficients and cycles."""
    rng = np.random.default_rng(3000 + seed)
    N = int(rng.choice([1, 3, 7, 15, 31, 63]))
    M = int(rng.integers(1, 300))
    alpha = float(rng.uniform(0.05, 1.0))
    cc, q = float(rng.uniform(0.0, 2.0)), float(rng.uniform(0.0, 2.0))
    nu1, nu2 = [int(v) for v in rng.integers(0, 3, size=2)]
    if nu1 + nu2 == 0:
        nu1 = 1
    first = int(rng.integers(0, 2))
    cycles = int(rng.integers(1, 3))
    f = rng.standard_normal((M, N))
    print(dict(N=N, M=M, alpha=alpha, c=cc, q=q, nu1=nu1, nu2=nu2, first=first, cycles=cycles), flush=True)
    ref, _ = oracle.nl_solve(N, M, alpha, f, c=cc, q=q, nu1=nu1, nu2=nu2, first=first, tol=1e-300, maxit=cycles)
    U = torch.zeros((M, N), dtype=torch.float64, device="cuda")
    info = B.fas_solve(dev(f), U, alpha, c=cc, q=q, nu1=nu1, nu2=nu2, first_colour=first, tol=1e-300, maxit=cycles)
    assert info["iters"] == cycles, info
    assert np.abs(host(U) - ref).max() <= 1e-11 * max(1.0, np.abs(ref).max())
