"""Seeded synthetic workloads for the time-fractional heat equation.

This module only synthesises inputs: forcing f sampled at the grid nodes, the
initial condition g, and the same forcing written as a short list of sine
modes with time profiles.  It holds none of the solver's arithmetic and
imports nothing from the rest of the package, so the GPU library's tests and
the CPU oracle can both take their inputs from it.

Grid conventions: interior nodes x_n = n h (n = 1..N, h = L/(N+1)), time
levels t_m = m tau (m = 1..M, tau = T/M); a grid function is [M, N] (1D) or
[M, N, N] (2D, x fastest) with row m-1 holding t_m.

Workloads (all on the unit interval / square, T = 1, zero initial data):
  * ``manufactured_1d``: u = t^2 sin(pi x), so f = (2 t^{2-a}/Gamma(3-a) +
    pi^2 t^2) sin(pi x) (the Caputo derivative of t^2 is 2 t^{2-a}/Gamma(3-a)).
  * ``random_modes_1d``: t^{1.5} sum_{k=1}^{20} (a_k/k^2) sin(k pi x), a_k ~
    N(0, 1) drawn from a seeded numpy Generator.
  * ``manufactured_2d``: u = t^2 sin(pi x) sin(pi y).
  * ``nonsmooth_2d``: u = (t^a + t^2) sin(pi x) sin(pi y), whose Caputo
    derivative has the constant part Gamma(1 + a).
  * ``batch_1d``: many 1D problems with N, M, alpha drawn from one seeded
    Generator and per-problem random-mode forcing.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field
from typing import List, Optional

import numpy as np

SEED = 1608


@dataclass
class Workload:
    """A problem instance: sizes, order, and the forcing as sine modes."""
    dims: int
    N: int
    M: int
    alpha: float
    T: float = 1.0
    L: float = 1.0
    kx: np.ndarray = field(default_factory=lambda: np.zeros(0, dtype=np.int32))
    ky: np.ndarray = field(default_factory=lambda: np.zeros(0, dtype=np.int32))
    s: np.ndarray = field(default_factory=lambda: np.zeros((0, 0)))  # [K, M] time profiles
    exact: Optional[object] = None  # callable u(x, t) or u(x, y, t) (continuous solution)
    name: str = ""

    @property
    def npts(self) -> int:
        return self.N if self.dims == 1 else self.N * self.N

    @property
    def unknowns(self) -> int:
        return self.npts * self.M

    def times(self) -> np.ndarray:
        return self.T * np.arange(1, self.M + 1, dtype=np.float64) / self.M

    def nodes(self) -> np.ndarray:
        return self.L * np.arange(1, self.N + 1, dtype=np.float64) / (self.N + 1)

    def mode_shapes(self) -> np.ndarray:
        """phi_q at the interior nodes: [K, N] (1D) or [K, N, N] (2D, x fastest)."""
        x = self.nodes()
        px = np.sin(np.pi * np.outer(self.kx, x) / self.L)
        if self.dims == 1:
            return px
        py = np.sin(np.pi * np.outer(self.ky, x) / self.L)
        return py[:, :, None] * px[:, None, :]

    def forcing(self) -> np.ndarray:
        """Dense f = sum_q s_q(t_m) phi_q(x_n) as a NumPy FP64 array."""
        ph = self.mode_shapes().reshape(len(self.kx), -1)
        f = self.s.T @ ph
        return f.reshape((self.M, self.N) if self.dims == 1 else (self.M, self.N, self.N))

    def forcing_torch(self, device):
        """Same forcing built with torch on ``device`` (for the large sizes)."""
        import torch
        ph = torch.from_numpy(np.ascontiguousarray(self.mode_shapes().reshape(len(self.kx), -1)))
        s = torch.from_numpy(np.ascontiguousarray(self.s))
        ph = ph.to(device)
        s = s.to(device)
        f = s.T.contiguous() @ ph
        return f.reshape((self.M, self.N) if self.dims == 1 else (self.M, self.N, self.N))

    def exact_grid(self) -> np.ndarray:
        t = self.times()
        x = self.nodes()
        if self.dims == 1:
            return self.exact(x[None, :], t[:, None])
        return self.exact(x[None, None, :], x[None, :, None], t[:, None, None])


def _caputo_t2(t, a):
    return 2.0 * t ** (2.0 - a) / math.gamma(3.0 - a)


def manufactured_1d(N=63, M=64, alpha=0.5, T=1.0) -> Workload:
    t = T * np.arange(1, M + 1) / M
    s = (_caputo_t2(t, alpha) + np.pi ** 2 * t ** 2)[None, :]
    return Workload(1, N, M, alpha, T, 1.0, np.array([1], np.int32), np.array([0], np.int32), s,
                    exact=lambda x, tt: tt ** 2 * np.sin(np.pi * x), name="manufactured_1d")


def random_mode_coeffs(seed: int, K: int = 20) -> np.ndarray:
    rng = np.random.default_rng(seed)
    a = rng.standard_normal(K)
    return a / np.arange(1, K + 1) ** 2


def random_modes_1d(N, M, alpha, seed=SEED, K=20, T=1.0, with_manufactured=False) -> Workload:
    t = T * np.arange(1, M + 1) / M
    coef = random_mode_coeffs(seed, K)
    s = np.outer(coef, t ** 1.5)
    kx = np.arange(1, K + 1, dtype=np.int32)
    exact = None
    if with_manufactured:
        s[0] += _caputo_t2(t, alpha) + np.pi ** 2 * t ** 2
    return Workload(1, N, M, alpha, T, 1.0, kx, np.zeros(K, np.int32), s, exact=exact,
                    name="random_modes_1d" + ("+manufactured" if with_manufactured else ""))


def config2(alpha=0.3, N=4095, M=16384) -> Workload:
    """1D, N = 4095, M = 16384: manufactured term plus seeded random modes."""
    w = random_modes_1d(N, M, alpha, seed=SEED, with_manufactured=True)
    w.name = f"1d_N{N}_M{M}_a{alpha}"
    return w


def manufactured_2d(N=511, M=2048, alpha=0.4, T=1.0) -> Workload:
    t = T * np.arange(1, M + 1) / M
    s = (_caputo_t2(t, alpha) + 2.0 * np.pi ** 2 * t ** 2)[None, :]
    return Workload(2, N, M, alpha, T, 1.0, np.array([1], np.int32), np.array([1], np.int32), s,
                    exact=lambda x, y, tt: tt ** 2 * np.sin(np.pi * x) * np.sin(np.pi * y),
                    name=f"2d_manufactured_N{N}_M{M}_a{alpha}")


def nonsmooth_2d(N=1023, M=1024, alpha=0.3, T=1.0) -> Workload:
    t = T * np.arange(1, M + 1) / M
    s = (math.gamma(1.0 + alpha) + _caputo_t2(t, alpha)
         + 2.0 * np.pi ** 2 * (t ** alpha + t ** 2))[None, :]
    return Workload(2, N, M, alpha, T, 1.0, np.array([1], np.int32), np.array([1], np.int32), s,
                    exact=lambda x, y, tt: (tt ** alpha + tt ** 2) * np.sin(np.pi * x) * np.sin(np.pi * y),
                    name=f"2d_nonsmooth_N{N}_M{M}_a{alpha}")


def batch_1d(count=256, seed=SEED, Ns=(127, 255, 511, 1023, 2047),
             Ms=(256, 512, 1024, 2048, 4096, 8192), alpha_range=(0.1, 0.9)) -> List[Workload]:
    """Many independent 1D problems of uneven (N, M, alpha)."""
    rng = np.random.default_rng(seed)
    Nl = rng.choice(np.asarray(Ns), size=count)
    Ml = rng.choice(np.asarray(Ms), size=count)
    al = rng.uniform(alpha_range[0], alpha_range[1], size=count)
    out = []
    for i in range(count):
        w = random_modes_1d(int(Nl[i]), int(Ml[i]), float(al[i]), seed=seed + 1 + i)
        w.name = f"batch{i}"
        out.append(w)
    return out


def paper_test1(N=127, M=128, alpha=0.4) -> Workload:
    """Section 7, first test problem: [0, pi] x [0, 1], f = 0, g = sin x."""
    w = Workload(1, N, M, alpha, 1.0, math.pi, np.array([1], np.int32), np.array([0], np.int32),
                 np.zeros((1, M)), name=f"paper_test1_N{N}_M{M}_a{alpha}")
    return w


def paper_test1_g(w: Workload) -> np.ndarray:
    return np.sin(w.nodes())


def paper_test2(N=31, M=32, alpha=0.4) -> Workload:
    """Section 7, second test problem on (0, 2)^2 with the forcing as printed,
    (2 t^{2-a}/Gamma(3-a) + (1 + pi^2/2) t^2) sin(pi x/2) sin(pi y/2).  The
    printed u = t^2 sin sin solves it only without the "1 +" term, so no
    continuous solution is attached; the iteration counts do not depend on it."""
    t = np.arange(1, M + 1) / M
    s = (_caputo_t2(t, alpha) + (1.0 + np.pi ** 2 / 2.0) * t ** 2)[None, :]
    return Workload(2, N, M, alpha, 1.0, 2.0, np.array([1], np.int32), np.array([1], np.int32), s,
                    exact=None, name=f"paper_test2_N{N}_M{M}_a{alpha}")
