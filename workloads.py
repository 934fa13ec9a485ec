"""Seeded synthetic inputs shared by the oracle side and the HIP side.

This module only draws random numbers; it holds none of the method's
arithmetic. Every array is produced by numpy ``Generator(PCG64(seed))`` so the
two sides always see bit-identical inputs.

The paper uses synthetic random point clouds only (Sec. 3.1: points on the
unit sphere and in a cube; Sec. 3.2: points uniform in a cube), so these
generators stand in for its workloads; no dataset is involved.

Workloads (names used across tests and the benchmark):

* ``uniform2d_2048``  N=2048 uniform in [0,1]^2, inverse multiquadric
  c=0.01 with 1.0 on the diagonal, quadtree depth 4, Chebyshev order 4,
  eps=1e-8, one N(0,1) right-hand side.
* ``uniform3d_65536`` N=65536 uniform in [0,1]^3, inverse multiquadric
  c=0.005 with 1.0 on the diagonal, octree depth 5, Chebyshev order 3,
  eps=1e-6, 16 N(0,1) right-hand sides.
* ``cluster3d_1m``    N=2^20, 8 Gaussian clusters (sigma 0.05, centres
  uniform in [0,1]^3), Gaussian kernel exp(-r^2/0.1^2) with 0.1 on the
  diagonal, octree depth 7, Chebyshev order 4; FP32 factors at eps=1e-5 vs
  FP64 factors at eps=1e-10.
* ``batch512``        512 problems, N log-uniform in [1024, 16384], even k on
  the unit sphere, odd k uniform in the unit cube, IMQ c=0.01 + 1.0 I,
  Chebyshev order 3, eps=1e-6, depth: smallest uniform depth >= 2 with at
  most 64 points per leaf.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np


def rng(seed: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(seed))


def uniform_cube(n: int, dim: int, seed: int) -> np.ndarray:
    """n points uniform in [0,1]^dim, float64, row-major (n, dim)."""
    return rng(seed).random((n, dim))


def unit_sphere(n: int, seed: int) -> np.ndarray:
    """n points uniform on the unit sphere surface in 3D (normalised Gaussians)."""
    g = rng(seed).standard_normal((n, 3))
    return g / np.linalg.norm(g, axis=1, keepdims=True)


def clustered(n_clusters: int, per_cluster: int, sigma: float, seed_centres: int,
              seed_points: int, dim: int = 3) -> np.ndarray:
    """Gaussian clusters: centres uniform in [0,1]^dim, points centre + sigma*N(0,I)."""
    centres = rng(seed_centres).random((n_clusters, dim))
    g = rng(seed_points).standard_normal((n_clusters, per_cluster, dim))
    pts = centres[:, None, :] + sigma * g
    return pts.reshape(n_clusters * per_cluster, dim)


def normal_rhs(n: int, nrhs: int, seed: int) -> np.ndarray:
    """Right-hand sides with i.i.d. N(0,1) entries, column-major (n, nrhs) Fortran order."""
    return np.asfortranarray(rng(seed).standard_normal((nrhs, n)).T)


@dataclass
class Workload:
    name: str
    points: np.ndarray          # (N, dim) float64
    kernel: str                 # "imq" | "gauss" | "paper" | "poly2"
    kparam: float               # c (imq), h (gauss), d (paper), unused (poly2)
    shift: float                # added on the diagonal of A
    depth: int                  # leaf level L
    order: int                  # Chebyshev nodes per dimension
    eps: float
    rhs: np.ndarray             # (N, nrhs) column-major
    extra: dict = field(default_factory=dict)

    @property
    def n(self) -> int:
        return self.points.shape[0]

    @property
    def dim(self) -> int:
        return self.points.shape[1]


def uniform2d_2048() -> Workload:
    pts = uniform_cube(2048, 2, 1001)
    return Workload("uniform2d_2048", pts, "imq", 0.01, 1.0, 4, 4, 1e-8,
                    normal_rhs(2048, 1, 1002))


def uniform3d_65536(n: int = 65536, depth: int = 5, nrhs: int = 16) -> Workload:
    pts = uniform_cube(n, 3, 2001)
    return Workload("uniform3d_%d" % n, pts, "imq", 0.005, 1.0, depth, 3, 1e-6,
                    normal_rhs(n, nrhs, 2002))


def cluster3d(n_per_cluster: int = 131072, depth: int = 7, eps: float = 1e-5) -> Workload:
    pts = clustered(8, n_per_cluster, 0.05, 3001, 3002)
    n = pts.shape[0]
    return Workload("cluster3d_%d" % n, pts, "gauss", 0.1, 0.1, depth, 4, eps,
                    normal_rhs(n, 1, 3003))


def batch_sizes(count: int = 512, lo: int = 1024, hi: int = 16384, seed: int = 4001) -> np.ndarray:
    u = rng(seed).random(count)
    return np.rint(np.exp(math.log(lo) + u * (math.log(hi) - math.log(lo)))).astype(np.int64)


def batch_problem(k: int, n: int) -> np.ndarray:
    return unit_sphere(n, 4100 + k) if k % 2 == 0 else uniform_cube(n, 3, 4100 + k)


def paper_cube(n: int = 100000, d: float = 1e-3, order: int = 3, depth: int = 3, eps: float = 1e-3,
               seed: int = 6001) -> Workload:
    """The paper's own GMRES workload (Sec. 3.2, Tables 1-2): n points uniform in [-1,1]^3, kernel
    K(0)=1, r/d below d, d/r above, no diagonal shift, eps 1e-3. The octree depth giving leaves closest to
    100 points is 3 for n = 1e5 (about 195 per leaf; depth 4 gives about 24). The solution x has
    N(0,1) entries (seed + 1); the right-hand side is formed from it by the caller's matvec."""
    pts = 2.0 * uniform_cube(n, 3, seed) - 1.0
    return Workload("paper_cube_%d_d%g_n%d" % (n, d, order), pts, "paper", d, 0.0, depth, order, eps,
                    normal_rhs(n, 1, seed + 1))


def small_uniform(n: int, dim: int, seed: int, depth: int, order: int, eps: float,
                  kernel: str = "imq", kparam: float = 0.01, shift: float = 1.0,
                  nrhs: int = 1) -> Workload:
    """Small problem of the same kind as the headline workloads, for tests."""
    return Workload("uniform%dd_%d_s%d" % (dim, n, seed), uniform_cube(n, dim, seed), kernel,
                    kparam, shift, depth, order, eps, normal_rhs(n, nrhs, seed + 1))


def small_cluster(n_per_cluster: int, seed: int, depth: int, order: int, eps: float,
                  nrhs: int = 1) -> Workload:
    pts = clustered(8, n_per_cluster, 0.05, seed, seed + 1)
    n = pts.shape[0]
    return Workload("cluster3d_%d_s%d" % (n, seed), pts, "gauss", 0.1, 0.1, depth, order, eps,
                    normal_rhs(n, nrhs, seed + 2))
