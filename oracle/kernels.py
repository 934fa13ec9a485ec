"""Matrix-entry kernels a_ij = K(|r_i - r_j|) (oracle; test infrastructure).

Sec. 2.1: A is given by a smooth kernel on a point cloud. Sec. 3.1 gives the
paper's own kernel: K(0) = 1, K(r) = r/d for 0 < r < d, K(r) = d/r otherwise.
The other kernels are those of the headline workloads (inverse multiquadric
and Gaussian) and a radial polynomial used only by tests, because Chebyshev
interpolation of order >= 3 reproduces it exactly.

Reading: a shift s is added on the diagonal of A only (a_ii = K(0) + s).
"""
from __future__ import annotations

import numpy as np

KINDS = {"imq": 0, "gauss": 1, "paper": 2, "poly2": 3}


def kernel_of_r(kind: str, param: float, r: np.ndarray) -> np.ndarray:
    r = np.asarray(r, dtype=np.float64)
    if kind == "imq":
        return 1.0 / np.sqrt(r * r + param * param)
    if kind == "gauss":
        return np.exp(-(r * r) / (param * param))
    if kind == "paper":
        out = np.empty_like(r)
        z = r == 0.0
        small = (r > 0.0) & (r < param)
        big = r >= param
        out[z] = 1.0
        out[small] = r[small] / param
        out[big] = param / r[big]
        return out
    if kind == "poly2":
        return 1.0 + r * r
    raise ValueError(kind)


def block(kind: str, param: float, X: np.ndarray, Y: np.ndarray) -> np.ndarray:
    """K(|x_a - y_b|) for all rows of X against all rows of Y (no shift)."""
    diff = X[:, None, :] - Y[None, :, :]
    r = np.sqrt(np.sum(diff * diff, axis=2))
    return kernel_of_r(kind, param, r)


def dense(kind: str, param: float, shift: float, P: np.ndarray) -> np.ndarray:
    """The dense matrix A of the point cloud P, with the diagonal shift."""
    A = block(kind, param, P, P)
    A[np.diag_indices_from(A)] += shift
    return A
