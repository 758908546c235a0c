"""Semi-algebraic mode analysis of the two-grid waveform-relaxation cycle
(Section 4): Fourier analysis in space, exact in time.

A low frequency theta (theta h in (0, pi/2]) and its high harmonic
theta - pi/h span a space that every operator of the 1D two-grid cycle maps
to itself.  Carried over the M time levels, each operator becomes a 2M x 2M
matrix whose time coupling is the lower-triangular Toeplitz matrix T_M of the
L1 scheme (Section 4.1):

* the red-black smoother: S = S_black S_red, each half-sweep coupling the two
  harmonics through the Jacobi-type splitting A_h = M_h - N_h, M_h = 2/h^2;
* the coarse-grid correction C = I - P (T_M + A_2h(2 theta))^-1 R A with
  full-weighting restriction and linear interpolation, both of symbol
  (1 + cos theta h) / 2, and A = diag(T_M + A_h(theta), T_M + A_h(theta - pi/h));
* the two-grid operator S^nu2 C S^nu1.

Only lambda = tau^alpha Gamma(2 - alpha) / h^2 matters, so the analysis takes
h = 1.  The predicted two-grid factor is the largest eigenvalue modulus over
a sample of theta.  The matrices are block lower triangular in time with the
same 2 x 2 block on the diagonal, so in exact arithmetic their spectral radius
is that block's and does not depend on M (``exact=True``); the factors
printed in the paper vary with M and are matched by the eigenvalues as
computed numerically (``exact=False``, the default), which for these
defective matrices are spread by rounding.

A CPU analysis tool of the method (numpy); not part of the solve path.  The
L1 coefficients come from the library's host code.
"""
import math

import numpy as np
from scipy import linalg

from . import binding


def time_matrix(M: int, alpha: float, lam: float) -> np.ndarray:
    """T_M of the L1 scheme for h = 1 and tau from lam = tau^alpha Gamma(2 - alpha)."""
    tau = (lam / math.gamma(2.0 - alpha)) ** (1.0 / alpha)
    _, r = binding.l1_weights(M, alpha, M * tau)
    return linalg.toeplitz(r, np.zeros(M))


def symbol_laplacian(theta: float) -> float:
    """Symbol of A_h = [-1 2 -1] / h^2 at theta h = theta (h = 1): 4 sin^2(theta / 2)."""
    return 4.0 * math.sin(0.5 * theta) ** 2


def two_grid_symbol(theta: float, Tm: np.ndarray, nu1: int = 1, nu2: int = 0) -> np.ndarray:
    """2M x 2M matrix of the two-grid operator on the harmonics (theta, theta - pi)."""
    M = Tm.shape[0]
    I = np.eye(M)
    t0, t1 = theta, theta - math.pi
    # one Jacobi-type step per harmonic: (T_M + M_h)^-1 N_h(theta), N_h = 2 cos(theta)
    Mt = Tm + 2.0 * I
    S0 = linalg.solve_triangular(Mt, 2.0 * math.cos(t0) * I, lower=True)
    S1 = linalg.solve_triangular(Mt, 2.0 * math.cos(t1) * I, lower=True)
    red = 0.5 * np.block([[S0 + I, S1 - I], [S0 - I, S1 + I]])
    black = 0.5 * np.block([[S0 + I, I - S1], [I - S0, S1 + I]])
    S = black @ red
    w0, w1 = 0.5 * (1.0 + math.cos(t0)), 0.5 * (1.0 + math.cos(t1))
    R = np.hstack([w0 * I, w1 * I])
    P = R.T
    A = np.block([[Tm + symbol_laplacian(t0) * I, 0 * I], [0 * I, Tm + symbol_laplacian(t1) * I]])
    Ac = Tm + 0.25 * symbol_laplacian(2.0 * t0) * I       # A_2h at 2 theta: 4 sin^2(theta) / (2h)^2
    C = np.eye(2 * M) - P @ linalg.solve_triangular(Ac, R @ A, lower=True)
    return np.linalg.matrix_power(S, nu2) @ C @ np.linalg.matrix_power(S, nu1)


def _radius(T: np.ndarray, exact: bool) -> float:
    if exact:   # block lower triangular in time: the first time level's 2 x 2 block
        M = T.shape[0] // 2
        return float(max(abs(np.linalg.eigvals(T[np.ix_([0, M], [0, M])]))))
    return float(max(abs(np.linalg.eigvals(T))))


def two_grid_factor(alpha: float, lam: float, M: int, nu1: int = 1, nu2: int = 0, ntheta: int = 64,
                    exact: bool = False) -> float:
    """Predicted two-grid factor: max over theta h in (0, pi/2] (ntheta samples)."""
    Tm = time_matrix(M, alpha, lam)
    thetas = np.linspace(math.pi / 2, 0.0, ntheta, endpoint=False)[::-1]
    return max(_radius(two_grid_symbol(t, Tm, nu1, nu2), exact) for t in thetas)
