"""Checkpoint/resume through warm_start and the failure paths a caller can
force from the host (through the C ABI)."""
import numpy as np
import pytest

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


@pytest.mark.parametrize("prec", ["fp64", "bf16x3"])
def test_warm_start_resumes_a_stopped_solve(B, prec):
    """Two cycles (stopped by maxit), then a warm-started solve from that
    iterate: its first residual is the stopped solve's last one, and it ends
    at the exact discrete solution."""
    w = W.random_modes_1d(127, 200, 0.4, seed=41)
    f = w.forcing()
    ref = oracle.direct_solve(1, w.N, w.M, w.alpha, f)
    with B.Solver(w.N, w.M, w.alpha, precision=prec, maxit=2) as s:
        U = torch.zeros(s.grid_shape, dtype=torch.float64, device="cuda")
        first = s.solve(dev(f), U, tol=1e-12, raise_on_error=False)
        assert first["rc"] == 1 and first["iters"] == 2, first   # MGWR_NOT_CONVERGED
        s.set_options(warm_start=1, maxit=100)
        second = s.solve(dev(f), U, tol=1e-12)
        torch.cuda.synchronize()
        U = U.cpu().numpy()
    # the checkpoint is the FP64 iterate u: in the refinement modes the low
    # part of the double-double iterate is not in it, which moves the residual
    # by A_h times a rounding of u (about 4/h^2 * eps * max|u|)
    h = 1.0 / (w.N + 1)
    slack = 0.0 if prec == "fp64" else 8.0 / h ** 2 * 2.3e-16 * float(np.abs(ref).max())
    assert abs(second["r0"] - first["rk"]) <= 1e-9 * first["rk"] + slack, (first, second)
    assert second["rc"] in (0, 2), second
    assert np.abs(U - ref).max() <= 1e-10 * np.abs(ref).max()


def test_absurd_size_is_out_of_memory(B):
    """A 2D hierarchy of 16383^2 points x 4096 levels (8.8 TB per grid
    function) fails cleanly with MGWR_ENOMEM."""
    with pytest.raises(B.MgwrError) as ei:
        B.Solver(16383, 4096, 0.5, dims=2)
    assert ei.value.code == -2, ei.value


def test_work_after_out_of_memory(B):
    """A failed allocation is reported by its call and leaves nothing behind:
    the next handle builds its coefficient tables (kernel launches checked
    with the runtime's last error) and solves."""
    with pytest.raises(B.MgwrError) as e:
        B.Solver(16383, 4096, 0.5, dims=2)
    assert e.value.code == B.MGWR_ENOMEM
    with B.Solver(15, 64, 0.5) as s:
        f = torch.ones((64, 15), dtype=torch.float64, device="cuda")
        U = torch.zeros_like(f)
        info = s.solve(f, U, tol=1e-10)
    assert info["status"] == "ok", info
