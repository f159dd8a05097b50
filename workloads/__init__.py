"""Seeded synthetic inputs for the space-fractional CGLE integrators.

This module only *describes* workloads: grid spacings, parameter sets and
initial conditions drawn from fixed seeds.  It holds none of the method's
arithmetic (no finite-difference weights, no eigendecomposition, no matrix
functions), so both the CPU oracle side and the HIP product side may take their
inputs from here without sharing any computation.

Grid (Section 2): n inner points x^j = a + j h, j = 1..n, h = (b - a)/(n + 1).
Tensors are C-ordered (n_1, ..., n_d) with axis d fastest.

The parameter sets and initial conditions follow the paper's Example 2 shape
(sech products with a phase, Section 4) extended to the workloads the
benchmarks run; every choice the paper leaves open is fixed here and listed
in the design notes.
"""
from __future__ import annotations

import dataclasses
from typing import List, Sequence, Tuple

import numpy as np

# (nu, eta, gamma, kappa, zeta) used by the 2-D parity workload and reused
# wherever a workload does not state its own set.
BASE_PARAMS = (1.0, 0.5, 1.0, 1.0, 0.5)


@dataclasses.dataclass
class Workload:
    name: str
    n: Tuple[int, ...]
    domain: Tuple[Tuple[float, float], ...]
    alpha: Tuple[float, ...]
    params: Tuple[float, float, float, float, float]
    tau: float
    steps: int
    scheme: str = "exp_euler"
    manufactured: bool = False

    @property
    def d(self) -> int:
        return len(self.n)

    @property
    def h(self) -> Tuple[float, ...]:
        return tuple((b - a) / (n + 1) for (a, b), n in zip(self.domain, self.n))

    def axes(self) -> List[np.ndarray]:
        return grid_axes(self.n, self.domain)


def grid_axes(n: Sequence[int], domain: Sequence[Tuple[float, float]]) -> List[np.ndarray]:
    """Inner grid points of each axis: x^j = a + j h, j = 1..n."""
    out = []
    for nm, (a, b) in zip(n, domain):
        h = (b - a) / (nm + 1)
        out.append(a + h * np.arange(1, nm + 1, dtype=np.float64))
    return out


def _mesh(axes: Sequence[np.ndarray]) -> List[np.ndarray]:
    return np.meshgrid(*axes, indexing="ij")


def sech_product(axes: Sequence[np.ndarray], k: Sequence[float], theta0: float = 0.0) -> np.ndarray:
    """u0 = prod_mu sech(x_mu) * exp(i (theta0 + sum_mu k_mu x_mu)), complex128, C-order."""
    X = _mesh(axes)
    amp = np.ones(X[0].shape)
    phase = np.full(X[0].shape, theta0)
    for xm, km in zip(X, k):
        amp = amp / np.cosh(xm)
        phase = phase + km * xm
    return (amp * np.exp(1j * phase)).astype(np.complex128)


def gaussian_sum(axes: Sequence[np.ndarray], seed: int = 21394, count: int = 4,
                 sigma: float = 1.0, centre_box: Tuple[float, float] = (-6.0, 6.0)) -> np.ndarray:
    """u0 = sum_k exp(i theta_k) exp(-|x - c_k|^2 / (2 sigma^2)), c_k ~ U(box)^d, theta_k ~ U(0, 2 pi).

    Draw order: c_1, theta_1, c_2, theta_2, ... from numpy default_rng(seed).
    """
    rng = np.random.default_rng(seed)
    X = _mesh(axes)
    d = len(axes)
    u = np.zeros(X[0].shape, np.complex128)
    for _ in range(count):
        c = rng.uniform(centre_box[0], centre_box[1], size=d)
        th = rng.uniform(0.0, 2.0 * np.pi)
        r2 = np.zeros(X[0].shape)
        for xm, cm in zip(X, c):
            r2 = r2 + (xm - cm) ** 2
        u = u + np.exp(1j * th) * np.exp(-r2 / (2.0 * sigma * sigma))
    return u


def random_complex(shape, seed: int, dtype=np.complex128) -> np.ndarray:
    """Standard complex normal entries, for operator-level parity tests."""
    rng = np.random.default_rng(seed)
    z = rng.standard_normal(shape) + 1j * rng.standard_normal(shape)
    return z.astype(dtype)


# --- the workloads -----------------------------------------------------------

def parity_2d() -> Workload:
    """2-D, 64x64 inner points on (-10,10)^2, alpha = (1.5, 1.5), 100 exp-Euler steps, tau = 1e-3."""
    return Workload("2d_64_expeuler", (64, 64), ((-10.0, 10.0),) * 2, (1.5, 1.5),
                    BASE_PARAMS, 1e-3, 100)


def u0_parity_2d(w: Workload) -> np.ndarray:
    return sech_product(w.axes(), (1.0, 0.0))


def manufactured_3d(scheme: str = "lbdf2", n: int = 128, steps: int = 1000, tau: float = 5e-4) -> Workload:
    """3-D 128^3 on (-8,8)^3, alpha = (1.3, 1.6, 1.8), manufactured u = e^{-t} prod sech(x_mu) e^{i x_1}."""
    return Workload(f"3d_{n}_manufactured_{scheme}", (n, n, n), ((-8.0, 8.0),) * 3, (1.3, 1.6, 1.8),
                    BASE_PARAMS, tau, steps, scheme=scheme, manufactured=True)


def u0_manufactured(w: Workload) -> np.ndarray:
    k = [1.0] + [0.0] * (w.d - 1)
    return sech_product(w.axes(), k)


def headline_3d(n: int = 256, steps: int = 200) -> Workload:
    """3-D 256^3 on (-12,12)^3, alpha = 1.7 per axis, 4 random Gaussians, 200 exp-Euler steps, tau = 1e-3."""
    return Workload(f"3d_{n}_gauss4_expeuler", (n, n, n), ((-12.0, 12.0),) * 3, (1.7, 1.7, 1.7),
                    BASE_PARAMS, 1e-3, steps)


def u0_headline(w: Workload) -> np.ndarray:
    return gaussian_sum(w.axes(), seed=21394)


def adjoint_3d(n: int = 96, steps: int = 200) -> Workload:
    """3-D 96^3 on (-10,10)^3, alpha = 1.5 per axis, 200 exp-Euler steps, tau = 1e-3."""
    return Workload(f"3d_{n}_adjoint", (n, n, n), ((-10.0, 10.0),) * 3, (1.5, 1.5, 1.5),
                    BASE_PARAMS, 1e-3, steps)


def strang_3d(n: int = 256, steps: int = 100, tau: float = 1e-2) -> Workload:
    """The paper's Example 2 in 3-D (Section 4, three-dimensional experiments): (-10,10)^3,
    alpha = (1.2, 1.8, 1.5),
    nu = eta = gamma = kappa = zeta = 1, no source, u0 = prod sech(x_mu) e^{i (x_1 + x_2 + x_3)};
    Strang splitting with tau = 1e-2 up to T = 1."""
    return Workload(f"3d_{n}_example2_strang", (n, n, n), ((-10.0, 10.0),) * 3, (1.2, 1.8, 1.5),
                    (1.0, 1.0, 1.0, 1.0, 1.0), tau, steps, scheme="strang")


def u0_strang(w: Workload) -> np.ndarray:
    return sech_product(w.axes(), [1.0] * w.d)


ADJOINT_PERTURBATION = (0.1, -0.1, 0.1, -0.1, 0.1)
ADJOINT_CHECKPOINT_EVERY = 20


def u0_adjoint(w: Workload) -> np.ndarray:
    return sech_product(w.axes(), [1.0] + [0.0] * (w.d - 1))


@dataclasses.dataclass
class BatchInstance:
    n: Tuple[int, int]
    alpha: Tuple[float, float]
    params: Tuple[float, float, float, float, float]
    theta0: float
    k: Tuple[float, float]
    domain: Tuple[Tuple[float, float], ...] = ((-10.0, 10.0), (-10.0, 10.0))

    @property
    def h(self) -> Tuple[float, float]:
        return tuple((b - a) / (n + 1) for (a, b), n in zip(self.domain, self.n))


def batch_2d(count: int = 64, seed: int = 2510, nmin: int = 96, nmax: int = 512) -> List[BatchInstance]:
    """Independent 2-D instances with uneven sizes and parameters.

    Per instance, in this order from default_rng(seed): n1, n2 ~ U{nmin..nmax},
    alpha_1, alpha_2 ~ U(1.2, 1.9), nu, kappa ~ U(0.5, 2), eta, zeta, gamma ~ U(-1, 1),
    theta0 ~ U(0, 2 pi), k_1, k_2 ~ U(-1, 1).
    """
    rng = np.random.default_rng(seed)
    out = []
    for _ in range(count):
        n1 = int(rng.integers(nmin, nmax + 1))
        n2 = int(rng.integers(nmin, nmax + 1))
        a1 = float(rng.uniform(1.2, 1.9))
        a2 = float(rng.uniform(1.2, 1.9))
        nu = float(rng.uniform(0.5, 2.0))
        kappa = float(rng.uniform(0.5, 2.0))
        eta = float(rng.uniform(-1.0, 1.0))
        zeta = float(rng.uniform(-1.0, 1.0))
        gamma = float(rng.uniform(-1.0, 1.0))
        th0 = float(rng.uniform(0.0, 2.0 * np.pi))
        k1 = float(rng.uniform(-1.0, 1.0))
        k2 = float(rng.uniform(-1.0, 1.0))
        out.append(BatchInstance((n1, n2), (a1, a2), (nu, eta, gamma, kappa, zeta), th0, (k1, k2)))
    return out


def u0_batch(inst: BatchInstance) -> np.ndarray:
    return sech_product(grid_axes(inst.n, inst.domain), inst.k, inst.theta0)


BATCH_TAU = 1e-3
BATCH_STEPS = 500
