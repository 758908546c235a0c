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
