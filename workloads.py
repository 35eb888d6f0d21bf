"""Seeded synthetic inputs shared by the tests, the benchmark and the oracle.

This module only draws random numbers.  It holds none of the method's
arithmetic (no kernel, no tree, no skeletonization), so both the HIP path and
the CPU oracle can take their inputs from it without sharing any code.

Every array is produced on the host in float64 with numpy's PCG64 generator.
Seeds follow one rule per workload number ``c`` (1 .. 6): points ``1000 + c``,
charges ``1100 + c``, target subset ``1200 + c``, weights ``1300 + c``; the
geometries of the batched workload (c = 5) add their index g as a second word
of the seed, ``[1000 + c, g]``.

The paper's experiments use synthetic point clouds (uniform square / cube,
sphere surface; section "Numerical results").  The workloads below take those
shapes at the sizes this library is measured on.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np


def _rng(seed) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(seed))


def uniform_points(n: int, dim: int, seed: int) -> np.ndarray:
    """n points iid uniform in the unit square / cube, shape (n, dim)."""
    return _rng(seed).random((n, dim))


def ellipsoid_points(n: int, seed: int, axes=(1.0, 0.5, 0.25), sigma=1e-3) -> np.ndarray:
    """Points on an ellipsoid surface, uniform in the surface parameters.

    theta ~ U[0, pi], phi ~ U[0, 2 pi); x = (a sin t cos p, b sin t sin p, c cos t),
    then displaced along the unit outward normal by xi ~ N(0, sigma).  Sampling
    uniform in (theta, phi) clusters points at the two z-poles, which makes the
    adaptive tree deep there.
    """
    g = _rng(seed)
    a, b, c = axes
    th = g.random(n) * math.pi
    ph = g.random(n) * (2.0 * math.pi)
    xi = g.standard_normal(n) * sigma
    st, ct, sp, cp = np.sin(th), np.cos(th), np.sin(ph), np.cos(ph)
    x = np.stack([a * st * cp, b * st * sp, c * ct], axis=1)
    nrm = np.stack([x[:, 0] / a**2, x[:, 1] / b**2, x[:, 2] / c**2], axis=1)
    nrm /= np.linalg.norm(nrm, axis=1, keepdims=True)
    return x + nrm * xi[:, None]


def charges(n: int, nrhs: int, seed: int, complex_: bool = False) -> np.ndarray:
    """Charges iid U[-1, 1]; shape (n,) for nrhs == 1 else (n, nrhs).

    Complex charges draw the real and imaginary parts independently.
    """
    g = _rng(seed)
    shape = (n,) if nrhs == 1 else (n, nrhs)
    if complex_:
        re = g.uniform(-1.0, 1.0, shape)
        im = g.uniform(-1.0, 1.0, shape)
        return re + 1j * im
    return g.uniform(-1.0, 1.0, shape)


def normal_weights(n: int, nrhs: int, seed: int) -> np.ndarray:
    g = _rng(seed)
    shape = (n,) if nrhs == 1 else (n, nrhs)
    return g.standard_normal(shape)


def target_subset(n: int, m: int, seed: int) -> np.ndarray:
    """m distinct target indices drawn without replacement, sorted."""
    m = min(m, n)
    return np.sort(_rng(seed).choice(n, size=m, replace=False)).astype(np.int64)


@dataclass
class Workload:
    """One synthetic workload: geometry, kernel, build parameters."""

    name: str
    number: int
    dim: int
    kind: str            # "laplace" or "helmholtz"
    n: int
    tol: float
    leaf_size: int
    geometry: str        # "uniform" or "ellipsoid"
    kappa: float = 0.0
    nrhs: int = 1
    complex_charges: bool = False
    n_targets: int = 2048
    extra: dict = field(default_factory=dict)
    index: int | None = None      # geometry index inside a batched workload

    def _seed(self, base: int):
        s = base + self.number
        return s if self.index is None else [s, self.index]

    def points(self) -> np.ndarray:
        seed = self._seed(1000)
        if self.geometry == "uniform":
            return uniform_points(self.n, self.dim, seed)
        if self.geometry == "ellipsoid":
            return ellipsoid_points(self.n, seed)
        raise ValueError(self.geometry)

    def charges(self, nrhs: int | None = None) -> np.ndarray:
        return charges(self.n, nrhs or self.nrhs, self._seed(1100), self.complex_charges)

    def targets(self, m: int | None = None) -> np.ndarray:
        return target_subset(self.n, m or self.n_targets, self._seed(1200))

    def weights(self, nrhs: int | None = None) -> np.ndarray:
        return normal_weights(self.n, nrhs or self.nrhs, self._seed(1300))


# 2D Laplace, N = 16,384 uniform in the unit square, leaf <= 64, tol 1e-8.
LAPLACE2D_16K = Workload("laplace2d_uniform_16k", 1, 2, "laplace", 16384, 1e-8, 64, "uniform")
# 3D Laplace, N = 2^20 uniform in the unit cube, leaf <= 128, tol 1e-7.
LAPLACE3D_1M = Workload("laplace3d_uniform_1m", 2, 3, "laplace", 1 << 20, 1e-7, 128, "uniform")
# 3D Laplace, N = 2^22 on the (1, 0.5, 0.25) ellipsoid surface, leaf <= 128, tol 1e-6.
LAPLACE3D_ELLIPSOID_4M = Workload("laplace3d_ellipsoid_4m", 3, 3, "laplace", 1 << 22, 1e-6, 128, "ellipsoid")
# 3D Helmholtz kappa = 20, N = 2^20 uniform, complex charges, leaf <= 128, tol 1e-6.
HELMHOLTZ3D_1M = Workload("helmholtz3d_k20_uniform_1m", 4, 3, "helmholtz", 1 << 20, 1e-6, 128, "uniform",
                          kappa=20.0, complex_charges=True)
# 2D Helmholtz kappa = 100 (the paper's 2D Helmholtz wavenumber), N = 16,384 uniform
# in the unit square, complex charges, leaf <= 64, tol 1e-8.
HELMHOLTZ2D_16K = Workload("helmholtz2d_k100_uniform_16k", 6, 2, "helmholtz", 16384, 1e-8, 64, "uniform",
                           kappa=100.0, complex_charges=True)


def batch_sizes(n_geom: int = 8, n_min: int = 65536, n_max: int = 2097152) -> list[int]:
    """Uneven geometry sizes growing geometrically from n_min to n_max."""
    ratio = n_max / n_min
    return [int(round(n_min * ratio ** (g / (n_geom - 1)))) for g in range(n_geom)]


def batch_workloads(n_geom: int = 8, sizes: list[int] | None = None, nrhs: int = 64) -> list[Workload]:
    """Eight 3D Laplace geometries alternating cube / ellipsoid, 64 RHS each."""
    sizes = sizes or batch_sizes(n_geom)
    out = []
    for g, n in enumerate(sizes):
        geo = "uniform" if g % 2 == 0 else "ellipsoid"
        out.append(Workload(f"batch_g{g}_{geo}_{n}", 5, 3, "laplace", n, 1e-6, 128, geo, nrhs=nrhs, index=g))
    return out


ALL = {w.name: w for w in (LAPLACE2D_16K, LAPLACE3D_1M, LAPLACE3D_ELLIPSOID_4M, HELMHOLTZ3D_1M, HELMHOLTZ2D_16K)}
