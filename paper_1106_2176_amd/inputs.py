"""Seeded synthetic workloads: uniformly random particles in a cube.

Every test problem of the paper is a set of uniformly random points in a cube
(captions of Fig. 4-9).  This module only draws random numbers; it holds none
of the method's arithmetic and is shared by the tests, the benchmark and the
CPU oracle's callers alike.

Generator: numpy PCG64 (``numpy.random.default_rng(seed)``).
  positions  U[0,1)^3 in FP64, cast (round to nearest even) to FP32 where the
             workload is FP32;
  charges    U[0,1), or U[-1,1) for the zero-mean workload;
  targets    ``default_rng(seed + 100).choice(N, n_targets, replace=False)``;
  weights    ``default_rng(seed + 200).standard_normal(N)`` (loss weights);
  clustered  Gaussian blobs for the adaptive tree (``clustered``).
"""
from dataclasses import dataclass

import numpy as np


@dataclass(frozen=True)
class Workload:
    name: str
    seed: int
    n: int
    p: int
    leaf_max: int
    charges: str  # "u01" or "u11"
    dtype: str    # "f64" or "f32"

    def describe(self) -> str:
        return (f"N={self.n:g} uniform cube, charges {'U[0,1)' if self.charges == 'u01' else 'U[-1,1)'}, "
                f"p={self.p}, leaf<={self.leaf_max}, {self.dtype} positions/charges")


# The five workloads of the benchmark plan (sizes, orders and leaf caps as
# stated there; seeds 1..5).
WORKLOADS = {
    "C1": Workload("C1", 1, 10_000, 4, 64, "u01", "f64"),
    "C2": Workload("C2", 2, 1_000_000, 10, 64, "u01", "f64"),
    "C3": Workload("C3", 3, 10_000_000, 10, 128, "u11", "f64"),
    "C4": Workload("C4", 4, 100_000_000, 8, 128, "u01", "f32"),
    "C5": Workload("C5", 5, 1_000_000, 8, 64, "u01", "f64"),
}


def particles(n: int, seed: int, charges: str = "u01", dtype: str = "f64"):
    """Positions [n,3] and charges [n] in the requested dtype."""
    rng = np.random.default_rng(seed)
    pos = rng.random((n, 3))
    if charges == "u01":
        q = rng.random(n)
    elif charges == "u11":
        q = rng.uniform(-1.0, 1.0, n)
    else:
        raise ValueError(charges)
    if dtype == "f32":
        return pos.astype(np.float32), q.astype(np.float32)
    return pos, q


def workload(name: str, n: int = None):
    """Positions and charges of a named workload (optionally with N overridden)."""
    w = WORKLOADS[name]
    return particles(n or w.n, w.seed, w.charges, w.dtype)


def targets(n: int, seed: int, n_targets: int = 1000) -> np.ndarray:
    """Sampled target indices for error checks."""
    k = min(n_targets, n)
    return np.sort(np.random.default_rng(seed + 100).choice(n, k, replace=False))


def weights(n: int, seed: int) -> np.ndarray:
    """Loss weights w ~ N(0,1) for the weighted-potential loss."""
    return np.random.default_rng(seed + 200).standard_normal(n)


def clustered(n: int, seed: int, blobs: int = 6, dtype: str = "f64"):
    """Positions [n,3] in Gaussian blobs and charges U[0,1) (inputs of the
    adaptive tree).  Blob centres U[0.2,0.8)^3, widths U[0.005,0.06), each
    particle in a uniformly chosen blob; coordinates clipped into [0,1)."""
    rng = np.random.default_rng(seed)
    cen = rng.uniform(0.2, 0.8, (blobs, 3))
    width = rng.uniform(0.005, 0.06, blobs)
    lab = rng.integers(0, blobs, n)
    pos = np.clip(cen[lab] + rng.normal(size=(n, 3)) * width[lab, None], 0.0, np.nextafter(1.0, 0.0))
    q = rng.random(n)
    if dtype == "f32":
        return pos.astype(np.float32), q.astype(np.float32)
    return pos, q
