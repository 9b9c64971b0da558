"""Seeded synthetic inputs shaped like the paper's regression and kriging workloads.

This module only draws inputs (points, targets, hyperparameters and solver
settings).  It contains none of the method's arithmetic and imports nothing
from the solver or from the oracle, so both may use it.

The paper's own datasets (the regression collection of section 6.1, the LIBSVM
sets of the Matern experiment and the Pacific-coast chlorophyll grid of the
kriging experiment) are not available; the recipes below stand in for their
shapes:

* ``plain_small`` (N=2000, d=2): the "2000 random points in a unit cube"
  convergence studies of section 5, drawn in two dimensions.
* ``kriging`` (N=1e5, d=3): a kriging-sized system (the paper's weekly kriging
  systems have about 1.8e5 points in d=3, section 6.3).
* ``clustered_large`` (N=1e6, d=2): beyond the paper's sizes; clustered points.
* ``batched``: 64 independent systems of uneven size, 16 right-hand sides each
  (the paper solves one kriging system per week).
* ``gp_regression`` (N=2e5, d=16): GP regression shaped like the larger
  regression datasets of Table 1.

Every generator uses numpy's PCG64 through ``default_rng(seed)``.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np


@dataclass
class Problem:
    """One regularised kernel system (K_hat + gamma I) w = y and its settings."""

    name: str
    x: np.ndarray            # (n, d) float64, C-contiguous
    y: np.ndarray            # (n,) or (n, nrhs) float64 (column-major RHS block: y[:, r])
    sigma: float
    gamma: float
    delta: float             # preconditioner shift: M = K_hat + delta I
    inner_maxit: int
    inner_tol: float
    tol: float = 1e-6
    restart: int = 30
    inner_prec: str = "fp32"
    extra: dict = field(default_factory=dict)

    @property
    def n(self) -> int:
        return int(self.x.shape[0])

    @property
    def d(self) -> int:
        return int(self.x.shape[1])


def _c(a: np.ndarray) -> np.ndarray:
    return np.ascontiguousarray(a, dtype=np.float64)


def plain_small(seed: int = 1, n: int = 2000) -> Problem:
    """N=2000, d=2, x ~ U[0,1]^2, y = sin(2 pi x1) cos(2 pi x2) + N(0, 0.01^2).

    sigma = 0.1, gamma = 1e-2.  Solved by plain FP64 CG and checked against a
    direct Cholesky solve; the mixed solver uses delta = 10 gamma with 10 inner
    iterations.
    """
    rng = np.random.default_rng(seed)
    x = rng.uniform(0.0, 1.0, size=(n, 2))
    y = np.sin(2 * np.pi * x[:, 0]) * np.cos(2 * np.pi * x[:, 1]) + 0.01 * rng.standard_normal(n)
    return Problem("plain_small", _c(x), _c(y), sigma=0.1, gamma=1e-2, delta=1e-1,
                   inner_maxit=10, inner_tol=1e-5)


def kriging(seed: int = 2, n: int = 100_000) -> Problem:
    """N=1e5, d=3, x ~ U[0,10]^3, y = sum of 64 random Fourier features + N(0, 0.05^2).

    Feature k is sqrt(2/64) cos(w_k . x + phi_k) with w_k ~ N(0, I_3) and
    phi_k ~ U[0, 2 pi].  sigma = 0.5, gamma = 1e-3; FGMRES with an FP64 outer MVP
    and exactly 10 FP32 inner CG iterations on K_hat + delta I, delta = 10 gamma.
    """
    rng = np.random.default_rng(seed)
    x = rng.uniform(0.0, 10.0, size=(n, 3))
    omega = rng.standard_normal((64, 3))
    phi = rng.uniform(0.0, 2 * np.pi, size=64)
    y = np.sqrt(2.0 / 64.0) * np.cos(x @ omega.T + phi).sum(axis=1) + 0.05 * rng.standard_normal(n)
    return Problem("kriging", _c(x), _c(y), sigma=0.5, gamma=1e-3, delta=1e-2,
                   inner_maxit=10, inner_tol=0.0)


def clustered_large(seed: int = 3, n: int = 1_000_000) -> Problem:
    """N=1e6, d=2: a 50-component Gaussian mixture with equal weights.

    Means ~ U[0,100]^2, standard deviations ~ U[0.5, 3], component ~ U{0..49};
    y = sin(2 pi x1 / 50) cos(2 pi x2 / 50) + N(0, 0.1^2).  sigma = 1, gamma = 1e-4,
    delta = 1e-3, BF16-input inner MVP, inner tolerance 1e-5, 10 inner iterations.
    """
    rng = np.random.default_rng(seed)
    means = rng.uniform(0.0, 100.0, size=(50, 2))
    stds = rng.uniform(0.5, 3.0, size=50)
    comp = rng.integers(0, 50, size=n)
    x = means[comp] + stds[comp, None] * rng.standard_normal((n, 2))
    y = np.sin(2 * np.pi * x[:, 0] / 50) * np.cos(2 * np.pi * x[:, 1] / 50) + 0.1 * rng.standard_normal(n)
    return Problem("clustered_large", _c(x), _c(y), sigma=1.0, gamma=1e-4, delta=1e-3,
                   inner_maxit=10, inner_tol=1e-5, inner_prec="bf16")


def batched(seed_base: int = 1000, nsys: int = 64, nrhs: int = 16,
            nmin: int = 1000, nmax: int = 50_000) -> list[Problem]:
    """64 independent systems; system k uses seed 1000+k.

    N_k ~ U{1000..50000}, d_k = 4 for even k and 8 for odd k, x ~ N(0, I),
    16 right-hand sides y ~ N(0, 1), sigma = sqrt(d_k), gamma = 1e-2; FP32 inner
    (delta = 0.1, 10 iterations), FP64 outer.
    """
    out = []
    for k in range(nsys):
        rng = np.random.default_rng(seed_base + k)
        n = int(rng.integers(nmin, nmax + 1))
        d = 4 if k % 2 == 0 else 8
        x = rng.standard_normal((n, d))
        y = np.asfortranarray(rng.standard_normal((n, nrhs)))
        out.append(Problem(f"batched[{k}]", _c(x), y, sigma=float(np.sqrt(d)), gamma=1e-2,
                           delta=1e-1, inner_maxit=10, inner_tol=0.0))
    return out


def gp_regression(seed: int = 5, n: int = 200_000, d: int = 16) -> Problem:
    """N=2e5, d=16, x ~ N(0, I), y = tanh(x . w) + N(0, 0.1^2) with w ~ N(0, I/d).

    sigma = 4, gamma = 1e-2 (the gradient workload).
    """
    rng = np.random.default_rng(seed)
    x = rng.standard_normal((n, d))
    wv = rng.standard_normal(d) / np.sqrt(d)
    y = np.tanh(x @ wv) + 0.1 * rng.standard_normal(n)
    return Problem("gp_regression", _c(x), _c(y), sigma=4.0, gamma=1e-2, delta=1e-1,
                   inner_maxit=10, inner_tol=1e-5)


def regression_highd(seed: int = 7, n: int = 44_484, d: int = 41) -> Problem:
    """GPR at the largest dimension and size of the regression table (d = 41,
    N = 44,484; the datasets themselves are absent and this stands in for their
    shape): x ~ N(0, I_d), y = tanh(x . w) + N(0, 0.1^2) with w ~ N(0, I/d);
    sigma = sqrt(d), gamma = 1e-2, delta = 10 gamma.
    """
    rng = np.random.default_rng(seed)
    x = rng.standard_normal((n, d))
    wv = rng.standard_normal(d) / np.sqrt(d)
    y = np.tanh(x @ wv) + 0.1 * rng.standard_normal(n)
    return Problem("regression_highd", _c(x), _c(y), sigma=float(np.sqrt(d)), gamma=1e-2, delta=1e-1,
                   inner_maxit=10, inner_tol=1e-5)


def matern_classification(seed: int = 6, n: int = 100_000, d: int = 8) -> Problem:
    """GPR on binary labels with the Matern-3/2 kernel (the classification sets of
    Table 2 are absent; this stands in for their shape at a larger N).

    x ~ N(0, I_d), labels y = sign(x . w + 0.3 e) in {-1, +1} with w ~ N(0, I/d),
    e ~ N(0, 1); length scale h = sqrt(d) (passed as sigma), gamma = 1e-2,
    delta = 10 gamma.
    """
    rng = np.random.default_rng(seed)
    x = rng.standard_normal((n, d))
    wv = rng.standard_normal(d) / np.sqrt(d)
    y = np.where(x @ wv + 0.3 * rng.standard_normal(n) >= 0.0, 1.0, -1.0)
    return Problem("matern_classification", _c(x), _c(y), sigma=float(np.sqrt(d)), gamma=1e-2, delta=1e-1,
                   inner_maxit=10, inner_tol=1e-5)


def random_points(seed: int, n: int, d: int, scale: float = 1.0, kind: str = "uniform") -> np.ndarray:
    """Plain random point sets for parity tests: uniform on [0, scale]^d or N(0, scale^2 I)."""
    rng = np.random.default_rng(seed)
    if kind == "uniform":
        x = rng.uniform(0.0, scale, size=(n, d))
    elif kind == "normal":
        x = scale * rng.standard_normal((n, d))
    else:
        raise ValueError(kind)
    return _c(x)


def random_vector(seed: int, n: int, nrhs: int | None = None) -> np.ndarray:
    """q ~ N(0, 1) (seeded); a column-major (n, nrhs) block when nrhs is given."""
    rng = np.random.default_rng(seed)
    if nrhs is None:
        return _c(rng.standard_normal(n))
    return np.asfortranarray(rng.standard_normal((n, nrhs)))


CONFIGS = {
    "plain_small": plain_small,
    "kriging": kriging,
    "clustered_large": clustered_large,
    "gp_regression": gp_regression,
}
