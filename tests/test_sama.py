"""Semi-algebraic mode analysis (Section 4): the predicted two-grid factors
against the paper's Table 2, and the 2M x 2M symbol against the two-grid
operator assembled as plain dense matrices on a periodic grid, where Fourier
modes are exact eigenfunctions.  CPU only."""
import math

import numpy as np
import pytest
from scipy import linalg

from conftest import load_golden
from paper_1608_05400_amd import sama


@pytest.mark.parametrize("row", load_golden("table2_wcycle_1d.txt"))
def test_table2_predicted_two_grid_factor(row):
    """Section 4, Table 2: alpha = 0.4, one pre-smoothing step; the predicted
    column, which the pseudospectral radius of the symbol at eps = u ||T||_2
    reproduces (the region where rounding puts the eigenvalues of these
    defective matrices; singular values do not depend on rounding details)."""
    l2lam, M, predicted, _measured = row
    rho = sama.two_grid_factor(0.4, 2.0 ** l2lam, int(M), reading="pseudospectral")
    assert abs(rho - predicted) <= 0.004, rho


@pytest.mark.parametrize("row", load_golden("table2_wcycle_1d.txt"))
def test_table2_measured_factor_is_the_finite_cycle_contraction(row):
    """Section 4, Table 2, the bracketed factors measured with the W-cycle:
    the two-grid contraction of M cycles, ||T^M||_2^(1/M), lies within 0.008
    of them, while the exact spectral radius does not depend on M."""
    l2lam, M, _predicted, measured = row
    q = sama.contraction(0.4, 2.0 ** l2lam, int(M), int(M), ntheta=16)
    rho = sama.two_grid_factor(0.4, 2.0 ** l2lam, int(M), reading="exact")
    assert abs(q - measured) <= 0.008, q
    assert rho <= q + 1e-12


@pytest.mark.parametrize("l2lam,M", [(0, 32), (2, 64)])
def test_numerical_eigenvalues_lie_in_the_pseudospectrum(l2lam, M):
    """The numerical reading, as a comparison: a backward-stable eigenvalue
    solver returns exact eigenvalues of T + E with ||E||_2 <= p(n) u ||T||_2,
    so their moduli lie between the exact radius and the pseudospectral
    radius at that eps (p(n) = 2n here)."""
    Tm = sama.time_matrix(M, 0.4, 2.0 ** l2lam)
    T = sama.two_grid_symbol(math.pi / 128, Tm)
    mu = sama._radius(T, True)
    num = sama._radius(T, False)
    eps = 2 * T.shape[0] * np.finfo(float).eps * np.linalg.norm(T, 2)
    ps = sama.pseudospectral_radius(T, eps, mu, phi0=math.pi)
    assert mu - 1e-12 <= num <= ps + 1e-12, (mu, num, ps)


def test_exact_radius_does_not_depend_on_M():
    """The symbol is block lower triangular in time with one 2 x 2 diagonal
    block: its exact spectral radius is that block's for every M, and at M = 1
    the numerical eigenvalues are exact."""
    r = [sama.two_grid_factor(0.4, 4.0, M, exact=True) for M in (1, 8, 32)]
    assert max(r) - min(r) <= 1e-12
    assert abs(sama.two_grid_factor(0.4, 4.0, 1) - r[0]) <= 1e-12


def test_laplacian_symbol_is_the_stencil_on_a_mode():
    x = np.arange(-3, 4)
    for theta in (0.3, 1.1, 2.9):
        phi = np.exp(1j * theta * x)
        Aphi = 2 * phi[3] - phi[2] - phi[4]
        assert abs(Aphi - sama.symbol_laplacian(theta) * phi[3]) <= 1e-13


def _periodic_two_grid(n, Tm, nu1, nu2, red_parity):
    """The two-grid error operator on n periodic points (h = 1) as a function
    on complex arrays e[m, j]: red-black sweeps (red = points of parity
    red_parity), full weighting, linear interpolation, exact coarse solve."""
    M = Tm.shape[0]
    Mt = Tm + 2.0 * np.eye(M)

    def A(e):
        return Tm @ e + 2.0 * e - np.roll(e, 1, axis=1) - np.roll(e, -1, axis=1)

    def half(e, parity):
        e = e.copy()
        for j in range(parity, n, 2):
            e[:, j] = linalg.solve_triangular(Mt, e[:, (j - 1) % n] + e[:, (j + 1) % n], lower=True)
        return e

    def sweep(e):
        return half(half(e, red_parity), 1 - red_parity)

    def restrict(r):
        return 0.25 * (np.roll(r, 1, axis=1) + 2.0 * r + np.roll(r, -1, axis=1))[:, 0::2]

    def prolong(ec):
        e = np.zeros((M, n), complex)
        e[:, 0::2] = ec
        e[:, 1::2] = 0.5 * (ec + np.roll(ec, -1, axis=1))
        return e

    def coarse_solve(rc):
        nc = rc.shape[1]
        Ac = np.kron(np.eye(nc), Tm) + np.kron(0.25 * (2.0 * np.eye(nc) - np.roll(np.eye(nc), 1, 0)
                                                       - np.roll(np.eye(nc), -1, 0)), np.eye(M))
        return np.linalg.solve(Ac, rc.T.reshape(-1)).reshape(nc, M).T

    def E(e):
        for _ in range(nu1):
            e = sweep(e)
        e = e - prolong(coarse_solve(restrict(A(e))))
        for _ in range(nu2):
            e = sweep(e)
        return e

    return E


@pytest.mark.parametrize("nu", [(1, 0), (1, 1), (0, 1)])
def test_symbol_matches_periodic_two_grid_operator(nu):
    n, M, alpha, lam = 16, 3, 0.6, 2.0
    Tm = sama.time_matrix(M, alpha, lam)
    E = _periodic_two_grid(n, Tm, nu[0], nu[1], red_parity=0)
    j = np.arange(n)
    for k in (1, 2, 3, 4):
        t0 = 2 * math.pi * k / n
        vs = [np.exp(1j * t0 * j), np.exp(1j * (t0 - math.pi) * j)]
        D = np.zeros((2 * M, 2 * M), complex)
        for a in range(2):
            for m in range(M):
                e = np.zeros((M, n), complex)
                e[m] = vs[a]
                out = E(e)
                for b in range(2):   # coordinates on the two harmonics
                    D[b * M:(b + 1) * M, a * M + m] = out @ vs[b].conj() / n
                # the pair of harmonics is invariant
                back = sum(np.outer(D[b * M:(b + 1) * M, a * M + m], vs[b]) for b in range(2))
                assert np.abs(out - back).max() <= 1e-12
        np.testing.assert_allclose(D, sama.two_grid_symbol(t0, Tm, nu[0], nu[1]), atol=1e-12)


def _periodic_two_grid_2d(n, Tm, nu1, nu2):
    """The 2D two-grid error operator on an n x n periodic grid (h = 1) as a
    function on complex arrays e[m, y, x]: red-black sweeps (red: x + y even,
    first), 9-point full weighting, bilinear interpolation, exact coarse solve."""
    M = Tm.shape[0]
    Mt = Tm + 4.0 * np.eye(M)

    def nbr(e):
        return (np.roll(e, 1, axis=2) + np.roll(e, -1, axis=2) + np.roll(e, 1, axis=1) + np.roll(e, -1, axis=1))

    def A(e, scale=1.0):
        return np.einsum("ab,byx->ayx", Tm, e) + scale * (4.0 * e - nbr(e))

    def half(e, parity):
        e = e.copy()
        for y in range(n):
            for x in range(n):
                if (x + y) % 2 == parity:
                    s = (e[:, y, (x - 1) % n] + e[:, y, (x + 1) % n] + e[:, (y - 1) % n, x] + e[:, (y + 1) % n, x])
                    e[:, y, x] = linalg.solve_triangular(Mt, s, lower=True)
        return e

    def sweep(e):
        return half(half(e, 0), 1)

    def restrict(r):
        rx = 0.25 * (np.roll(r, 1, axis=2) + 2.0 * r + np.roll(r, -1, axis=2))
        rxy = 0.25 * (np.roll(rx, 1, axis=1) + 2.0 * rx + np.roll(rx, -1, axis=1))
        return rxy[:, 0::2, 0::2]

    def prolong(ec):
        ex = np.zeros((M, ec.shape[1], n), complex)
        ex[:, :, 0::2] = ec
        ex[:, :, 1::2] = 0.5 * (ec + np.roll(ec, -1, axis=2))
        e = np.zeros((M, n, n), complex)
        e[:, 0::2, :] = ex
        e[:, 1::2, :] = 0.5 * (ex + np.roll(ex, -1, axis=1))
        return e

    def coarse_solve(rc):
        nc = rc.shape[1]
        cols = []
        for k in range(M * nc * nc):   # the coarse operator T_M + A_2h as a dense matrix
            u = np.zeros(M * nc * nc)
            u[k] = 1.0
            cols.append(A(u.reshape(M, nc, nc), 0.25).reshape(-1))
        return np.linalg.solve(np.array(cols).T, rc.reshape(-1)).reshape(rc.shape)

    def E(e):
        for _ in range(nu1):
            e = sweep(e)
        e = e - prolong(coarse_solve(restrict(A(e))))
        for _ in range(nu2):
            e = sweep(e)
        return e

    return E


@pytest.mark.parametrize("nu", [(1, 0), (1, 1)])
def test_symbol_2d_matches_periodic_two_grid_operator(nu):
    n, M, alpha, lam = 8, 2, 0.4, 1.5
    Tm = sama.time_matrix(M, alpha, lam)
    E = _periodic_two_grid_2d(n, Tm, nu[0], nu[1])
    y, x = np.meshgrid(np.arange(n), np.arange(n), indexing="ij")
    for kx, ky in ((1, 1), (1, 2), (2, 1)):
        tx, ty = 2 * math.pi * kx / n, 2 * math.pi * ky / n
        hs = [(tx, ty), (tx - math.pi, ty - math.pi), (tx - math.pi, ty), (tx, ty - math.pi)]
        vs = [np.exp(1j * (a * x + b * y)) for a, b in hs]
        D = np.zeros((4 * M, 4 * M), complex)
        for a in range(4):
            for m in range(M):
                e = np.zeros((M, n, n), complex)
                e[m] = vs[a]
                out = E(e)
                for b in range(4):
                    D[b * M:(b + 1) * M, a * M + m] = np.einsum("myx,yx->m", out, vs[b].conj()) / n ** 2
                back = sum(np.einsum("m,yx->myx", D[b * M:(b + 1) * M, a * M + m], vs[b]) for b in range(4))
                assert np.abs(out - back).max() <= 1e-12
        np.testing.assert_allclose(D, sama.two_grid_symbol_2d(tx, ty, Tm, nu[0], nu[1]), atol=1e-12)


def test_2d_factors_bounded():
    """Section 6: the 2D two-grid factors for one smoothing step stay below
    0.25 over lambda and the fractional order (the exact radius, which does
    not depend on M)."""
    rho = {(alpha, l2): sama.two_grid_factor_2d(alpha, 2.0 ** l2, 4, ntheta=12, exact=True)
           for alpha in (0.1, 0.5, 0.9) for l2 in (-8, -4, 0, 4, 8)}
    assert max(rho.values()) <= 0.25, rho
    # and, against lambda = tau^alpha Gamma(2 - alpha) / h^2, they hardly
    # depend on the fractional order
    for l2 in (-8, -4, 0, 4, 8):
        assert max(abs(rho[(a, l2)] - rho[(0.5, l2)]) for a in (0.1, 0.9)) <= 0.01


def test_jacobi_smoothing_factor_closed_form():
    """Section 4.1: (T_M + 2)^-1 N(theta) is lower triangular with diagonal
    2 cos(theta) / (r_1 + 2), r_1 = 1/lambda for h = 1, so the exact factor
    over the high frequencies is 2 / (1/lambda + 2) (at theta h = pi)."""
    for lam in (0.25, 1.0, 16.0):
        mu = sama.smoothing_factor(0.4, lam, 16, exact=True)
        assert abs(mu - 2.0 / (1.0 / lam + 2.0)) <= 1e-13, (lam, mu)


def test_steady_limits():
    """Section 6 remark: as lambda grows the problem tends to the steady one,
    where red-black two-grid with full weighting and linear interpolation is
    exact in 1D and has the factor 1/4 in 2D (one smoothing step)."""
    assert sama.two_grid_factor(0.5, 2.0 ** 20, 4, exact=True) <= 1e-4
    assert abs(sama.two_grid_factor_2d(0.5, 2.0 ** 20, 2, ntheta=24, exact=True) - 0.25) <= 0.01
