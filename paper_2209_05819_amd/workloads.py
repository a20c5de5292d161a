"""Seeded synthetic workloads shaped like the paper's experiments.

This module only draws random numbers (NumPy PCG64); it holds none of the
method's arithmetic, so both the GPU library's tests and the CPU oracle's
tests take their inputs from it.

The paper's experiments use uniformly distributed particles in a hyper-cube
(sec. 6.1: [-1,1]^4; sec. 6.2: a uniform 4D grid) and clustered synthetic
data for the kernel SVM (sec. 6.3).  The named workloads below follow those
shapes at the sizes this library is measured on.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np


def rng(seed: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(seed))


def uniform_points(n: int, d: int, seed: int, lo: float = -1.0, hi: float = 1.0) -> np.ndarray:
    return rng(seed).uniform(lo, hi, size=(n, d))


def gaussian_mixture(n: int, d: int, seed: int, centres: int = 8, sigma: float = 0.1) -> np.ndarray:
    g = rng(seed)
    c = g.uniform(-1.0, 1.0, size=(centres, d))
    lab = g.integers(0, centres, size=n)
    return c[lab] + sigma * g.standard_normal(size=(n, d))


def interior_grid(n: int, d: int, lo: float = 0.0, hi: float = 1.0) -> np.ndarray:
    """n^d points lo + (hi-lo) k/(n+1), k = 1..n per axis (strictly interior)."""
    t = lo + (hi - lo) * np.arange(1, n + 1) / (n + 1)
    mesh = np.meshgrid(*([t] * d), indexing="ij")
    return np.stack([m.reshape(-1) for m in mesh], axis=1)


def rhs_uniform(n: int, nrhs: int, seed: int) -> np.ndarray:
    x = rng(seed).uniform(-1.0, 1.0, size=(nrhs, n)).T
    return np.asfortranarray(x)


def rhs_normal(n: int, nrhs: int, seed: int) -> np.ndarray:
    x = rng(seed).standard_normal(size=(nrhs, n)).T
    return np.asfortranarray(x)


@dataclass
class Workload:
    name: str
    N: int
    d: int
    kernel: str            # log | inv_r | inv_r2 | gauss | exp | r | sin | inv_sqrt1p
    h: float
    diag: float
    leaf: int
    tol: float
    nrhs: int
    point_seed: int
    rhs_seed: int
    dist: str              # uniform | mixture
    rhs_dist: str          # uniform | normal
    domain: tuple | None   # (lo vector, side) or None = bounding cube
    extra: dict = field(default_factory=dict)

    def points(self) -> np.ndarray:
        if self.dist == "uniform":
            return uniform_points(self.N, self.d, self.point_seed)
        return gaussian_mixture(self.N, self.d, self.point_seed)

    def rhs(self) -> np.ndarray:
        if self.rhs_dist == "uniform":
            return rhs_uniform(self.N, self.nrhs, self.rhs_seed)
        return rhs_normal(self.N, self.nrhs, self.rhs_seed)


def _cube(d):
    return (np.full(d, -1.0), 2.0)


WORKLOADS = {
    # 2D, log r (diag 0), leaf 64, ACA 1e-8: the small case the oracle checks in seconds
    "uniform2d_log_n4096": Workload("uniform2d_log_n4096", 4096, 2, "log", 1.0, 0.0, 64, 1e-8,
                                    1, 1, 101, "uniform", "uniform", _cube(2)),
    # 3D, 1/r (diag 0), leaf 64, ACA 1e-10: the throughput workload
    "uniform3d_invr_n262144": Workload("uniform3d_invr_n262144", 1 << 18, 3, "inv_r", 1.0, 0.0,
                                       64, 1e-10, 1, 2, 102, "uniform", "normal", _cube(3)),
    # 4D, 1/r^2 (diag 0), leaf 128, ACA 1e-8, 32 right-hand sides
    "uniform4d_invr2_n524288": Workload("uniform4d_invr2_n524288", 1 << 19, 4, "inv_r2", 1.0,
                                        0.0, 128, 1e-8, 32, 3, 103, "uniform", "normal",
                                        _cube(4)),
    # 3D Gaussian-mixture cloud, Gram matrix exp(-r^2/0.25) + 1e-3 I, 16 right-hand sides
    "mixture3d_gauss_n1048576": Workload("mixture3d_gauss_n1048576", 1 << 20, 3, "gauss", 0.5,
                                         1.0 + 1e-3, 64, 1e-6, 16, 4, 104, "mixture", "normal",
                                         None),
}


def scaled(w: Workload, N: int, **kw) -> Workload:
    """Same workload recipe at another size (for parity tests)."""
    d = dict(w.__dict__)
    d.update(kw)
    d["N"] = N
    d["name"] = f"{w.name}@{N}"
    return Workload(**d)
