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
is that block's and does not depend on M (``reading="exact"``).  The factors
printed in the paper vary with M.  They are the eigenvalues as computed
numerically (``reading="numerical"``), which for these defective matrices
are spread by rounding, and lie where rounding can put them: in the
eps-pseudospectrum for eps = u ||T||_2 (u = 2^-52), whose radius
(``reading="pseudospectral"``, the default) reproduces them
deterministically.  ``contraction`` gives the finite-k mean contraction
||T^k||_2^(1/k) of k two-grid cycles, the quantity an experiment of k cycles
measures.

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


def smoothing_factor(alpha: float, lam: float, M: int, ntheta: int = 64, exact: bool = False) -> float:
    """Smoothing factor of the Jacobi-type waveform relaxation (M_h = 2/h^2,
    the diagonal of A_h): the largest eigenvalue modulus of
    (T_M + M_h)^-1 N_h(theta) over the high frequencies theta h in [pi/2, pi]
    (Section 4.1, smoothing analysis)."""
    Tm = time_matrix(M, alpha, lam)
    Mt = Tm + 2.0 * np.eye(M)
    best = 0.0
    for t in np.linspace(math.pi / 2, math.pi, ntheta):
        S = linalg.solve_triangular(Mt, 2.0 * math.cos(t) * np.eye(M), lower=True)
        v = abs(S[0, 0]) if exact else float(max(abs(np.linalg.eigvals(S))))
        best = max(best, v)
    return best


def _radius(T: np.ndarray, exact: bool) -> float:
    if exact:   # block lower triangular in time: the first time level's 2 x 2 block
        M = T.shape[0] // 2
        return float(max(abs(np.linalg.eigvals(T[np.ix_([0, M], [0, M])]))))
    return float(max(abs(np.linalg.eigvals(T))))


def pseudospectral_radius(T: np.ndarray, eps: float, r0: float, nphi: int = 36, iters: int = 30,
                          phi0: float = 0.0) -> float:
    """Radius of the eps-pseudospectrum {z : sigma_min(T - z I) <= eps}
    reached along nphi directions (starting at angle phi0), by bisection on
    |z| from r0 (a point of the set, such as the modulus of an eigenvalue in
    direction phi0) to ||T||_2.  Singular values are perfectly conditioned,
    so the result does not depend on rounding details."""
    n = T.shape[0]
    eye = np.eye(n)
    phis = phi0 + 2.0 * math.pi * np.arange(nphi) / nphi

    def inside(r):
        return any(linalg.svdvals(T - r * np.exp(1j * p) * eye)[-1] <= eps for p in phis)

    lo, hi = r0, float(np.linalg.norm(T, 2))
    for _ in range(iters):
        mid = 0.5 * (lo + hi)
        if inside(mid):
            lo = mid
        else:
            hi = mid
    return lo


def two_grid_factor(alpha: float, lam: float, M: int, nu1: int = 1, nu2: int = 0, ntheta: int = 64,
                    exact: bool = False, reading: str = None) -> float:
    """Predicted two-grid factor, max over theta h in (0, pi/2] (ntheta
    samples): the exact spectral radius ("exact"), the largest modulus of the
    numerically computed eigenvalues ("numerical"), or the eps-pseudospectral
    radius for eps = u ||T||_2 ("pseudospectral", the default; evaluated at the
    sample where the exact radius is largest: both decrease with theta)."""
    reading = reading or ("exact" if exact else "pseudospectral")
    Tm = time_matrix(M, alpha, lam)
    thetas = np.linspace(math.pi / 2, 0.0, ntheta, endpoint=False)[::-1]
    if reading in ("exact", "numerical"):
        return max(_radius(two_grid_symbol(t, Tm, nu1, nu2), reading == "exact") for t in thetas)
    if reading != "pseudospectral":
        raise ValueError(f"unknown reading {reading}")
    syms = [two_grid_symbol(t, Tm, nu1, nu2) for t in thetas]
    blocks = [np.linalg.eigvals(T[np.ix_([0, M], [0, M])]) for T in syms]
    i = int(np.argmax([max(abs(w)) for w in blocks]))
    mu = blocks[i][np.argmax(abs(blocks[i]))]
    T = syms[i]
    eps = np.finfo(float).eps * np.linalg.norm(T, 2)
    return pseudospectral_radius(T, eps, abs(mu), phi0=float(np.angle(mu)))


def contraction(alpha: float, lam: float, M: int, k: int, nu1: int = 1, nu2: int = 0, ntheta: int = 64) -> float:
    """Mean contraction of k two-grid cycles, max over theta of ||T^k||_2^(1/k)."""
    Tm = time_matrix(M, alpha, lam)
    thetas = np.linspace(math.pi / 2, 0.0, ntheta, endpoint=False)[::-1]
    return max(np.linalg.norm(np.linalg.matrix_power(two_grid_symbol(t, Tm, nu1, nu2), k), 2) ** (1.0 / k)
               for t in thetas)


# ---------------------------------------------------------------------------
# 2D (Section 6): the four harmonics theta^00, theta^11, theta^10, theta^01
# (theta^ab = theta - (a pi, b pi)) of a low frequency theta in (0, pi/2]^2
# span an invariant space; the operators become 4M x 4M matrices.  The red-
# black mask e^{i pi (x + y)} pairs theta^00 with theta^11 and theta^10 with
# theta^01, so each half-sweep acts on those pairs as in 1D, with the
# splitting M_h = 4/h^2, N_h(theta) = 2 cos theta_x + 2 cos theta_y.

def _harmonics_2d(tx: float, ty: float):
    return [(tx, ty), (tx - math.pi, ty - math.pi), (tx - math.pi, ty), (tx, ty - math.pi)]


def symbol_laplacian_2d(tx: float, ty: float) -> float:
    """Symbol of the 5-point A_h (h = 1): 4 sin^2(theta_x / 2) + 4 sin^2(theta_y / 2)."""
    return symbol_laplacian(tx) + symbol_laplacian(ty)


def two_grid_symbol_2d(tx: float, ty: float, Tm: np.ndarray, nu1: int = 1, nu2: int = 0) -> np.ndarray:
    """4M x 4M matrix of the 2D two-grid operator on the harmonics of (tx, ty)."""
    M = Tm.shape[0]
    I = np.eye(M)
    Z = np.zeros((M, M))
    hs = _harmonics_2d(tx, ty)
    Mt = Tm + 4.0 * I
    Sj = [linalg.solve_triangular(Mt, (2.0 * math.cos(a) + 2.0 * math.cos(b)) * I, lower=True) for a, b in hs]

    def half(red: bool) -> np.ndarray:
        out = np.zeros((4 * M, 4 * M))
        s = 1.0 if red else -1.0
        for a, b in ((0, 1), (2, 3)):   # pairs coupled by the colour mask
            ia, ib = slice(a * M, (a + 1) * M), slice(b * M, (b + 1) * M)
            out[ia, ia] = 0.5 * (Sj[a] + I)
            out[ib, ib] = 0.5 * (Sj[b] + I)
            out[ia, ib] = 0.5 * s * (Sj[b] - I)
            out[ib, ia] = 0.5 * s * (Sj[a] - I)
        return out

    S = half(False) @ half(True)
    w = [0.25 * (1.0 + math.cos(a)) * (1.0 + math.cos(b)) for a, b in hs]
    R = np.hstack([wk * I for wk in w])
    P = R.T
    A = np.block([[Tm + symbol_laplacian_2d(*hs[k]) * I if k == l else Z for l in range(4)] for k in range(4)])
    Ac = Tm + 0.25 * symbol_laplacian_2d(2.0 * tx, 2.0 * ty) * I
    C = np.eye(4 * M) - P @ linalg.solve_triangular(Ac, R @ A, lower=True)
    return np.linalg.matrix_power(S, nu2) @ C @ np.linalg.matrix_power(S, nu1)


def _radius_blocks(T: np.ndarray, nb: int, exact: bool) -> float:
    if exact:
        M = T.shape[0] // nb
        idx = [k * M for k in range(nb)]
        return float(max(abs(np.linalg.eigvals(T[np.ix_(idx, idx)]))))
    return float(max(abs(np.linalg.eigvals(T))))


def two_grid_factor_2d(alpha: float, lam: float, M: int, nu1: int = 1, nu2: int = 0, ntheta: int = 16,
                       exact: bool = False) -> float:
    """Predicted 2D two-grid factor: max over (theta_x, theta_y) h in (0, pi/2]^2
    (ntheta samples per direction)."""
    Tm = time_matrix(M, alpha, lam)
    ts = np.linspace(math.pi / 2, 0.0, ntheta, endpoint=False)[::-1]
    return max(_radius_blocks(two_grid_symbol_2d(a, b, Tm, nu1, nu2), 4, exact) for a in ts for b in ts)
