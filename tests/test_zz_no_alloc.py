"""The allocation-free entry point mgwr_toeplitz_apply_static against
mgwr_toeplitz_apply: the same Toeplitz products (T_M, or the inverse of
T_M + sigma_l I on a level; Section 5 and Section 5.2) with every buffer
beyond B and C in the per-GPU static scratch.  Two calls in a row on one
handle, the second with fewer columns (the scratch keeps the first call's
contents), by both routes and in the three arithmetics, each checked against
the allocating entry point and against T @ X of the oracle's coefficients at
the product tolerances of the parity tests (FP64 1e-13, FP32 1e-6, split
BF16 5e-5 of the term size).  Sizes beyond the scratch are refused before
anything is launched."""
import numpy as np
import pytest
from scipy import linalg

import oracle

torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu

TOL = {"fp64": 1e-13, "fp32": 1e-6, "bf16x3": 5e-5}


@pytest.fixture(scope="module")
def B():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1608_05400_amd import binding
    binding.load()
    return binding


def _column(M, alpha, N, which, nlev):
    c, d, r = oracle.l1_coeffs(M, alpha)
    T = linalg.toeplitz(r, np.zeros_like(r))
    if which < 0:
        return T
    n = 2 ** (which + 1) - 1
    sigma = 2.0 * (n + 1) ** 2
    return linalg.solve_triangular(T + sigma * np.eye(M), np.eye(M), lower=True)


@pytest.mark.parametrize("prec", ["fp64", "fp32", "bf16x3"])
@pytest.mark.parametrize("fft", [0, 2])
@pytest.mark.parametrize("which", [-1, 3])
def test_static_matches_allocating_entry_point(B, prec, fft, which):
    M, N, alpha = 1000, 63, 0.45
    with B.Solver(N, M, alpha, dims=1, precision=prec, fft=fft) as s:
        X_full = _column(M, alpha, N, which, s.levels())
        for call, P in enumerate((700, 130)):   # the second call smaller
            rng = np.random.default_rng(10 * call + P)
            X = rng.standard_normal((M, P))
            Xd = torch.from_numpy(X).cuda()
            ref_dev = s.toeplitz_apply(Xd, which=which, precision=prec)
            C = torch.full_like(Xd, float("nan"))
            s.toeplitz_apply_static(Xd, which=which, precision=prec, C=C)
            torch.cuda.synchronize()
            got, ref_dev = C.cpu().numpy(), ref_dev.cpu().numpy()
            ref = X_full @ X
            scale = (np.abs(X_full) @ np.abs(X)).max()
            print(f"{prec} fft {fft} which {which} call {call} P {P}: "
                  f"vs entry point {np.abs(got - ref_dev).max() / scale:.2e} "
                  f"(bitwise {np.array_equal(got, ref_dev)}), vs T X {np.abs(got - ref).max() / scale:.2e}")
            assert np.isfinite(got).all()
            # the same launches (the split-K partials fit the scratch, so the
            # K splits are the allocating entry point's): the same bits
            assert np.array_equal(got, ref_dev)
            assert np.abs(got - ref_dev).max() <= TOL[prec] * scale
            assert np.abs(got - ref).max() <= TOL[prec] * scale


@pytest.mark.parametrize("prec,P", [("fp32", 4097), ("bf16x3", 4097)])
def test_static_refuses_operands_beyond_the_scratch(B, prec, P):
    """4 M P bytes of FP32 operand, or 4 Mpad ldp of split BF16, above
    MGWR_STATIC_SCRATCH_BYTES (64 MiB) for M = 4096: refused, C untouched."""
    M = 4096
    with B.Solver(7, M, 0.5, dims=1, precision=prec, fft=0) as s:
        X = torch.ones((M, P), dtype=torch.float64, device="cuda")
        C = torch.zeros_like(X)
        with pytest.raises(B.MgwrError) as e:
            s.toeplitz_apply_static(X, which=-1, precision=prec, C=C)
        assert e.value.code == B.MGWR_EINVAL
        assert "static scratch" in str(e.value)
        torch.cuda.synchronize()
        assert float(C.abs().max()) == 0.0
