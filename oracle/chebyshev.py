"""Chebyshev interpolation used to build the H2 operators (oracle; test infrastructure).

Sec. 3 opening: the initial low-rank approximations come from interpolation
based on Chebyshev polynomials, as in the black-box FMM of Fong and Darve.
Reading: first-kind nodes t_k = cos((2k-1) pi / (2n)), k = 1..n, and the
Lagrange basis on them, in tensor form over the d dimensions; the flat index
of a tensor node m = (m_0, ..., m_{d-1}) is sum_k m_k n^k.
"""
from __future__ import annotations

import itertools

import numpy as np


def nodes(n: int) -> np.ndarray:
    k = np.arange(1, n + 1, dtype=np.float64)
    return np.cos((2.0 * k - 1.0) * np.pi / (2.0 * n))


def lagrange_1d(n: int, x: np.ndarray) -> np.ndarray:
    """L[a, m] = prod_{k != m} (x_a - t_k) / (t_m - t_k), written out term by term."""
    t = nodes(n)
    x = np.asarray(x, dtype=np.float64)
    out = np.ones((x.shape[0], n))
    for m in range(n):
        for k in range(n):
            if k != m:
                out[:, m] *= (x - t[k]) / (t[m] - t[k])
    return out


def multi_indices(n: int, d: int) -> np.ndarray:
    """(n^d, d) tensor indices, dimension 0 varying fastest."""
    idx = np.array(list(itertools.product(range(n), repeat=d)))[:, ::-1]
    return np.ascontiguousarray(idx)


def lagrange_nd(n: int, X: np.ndarray) -> np.ndarray:
    """Tensor Lagrange basis at reference points X (M, d) in [-1,1]^d -> (M, n^d)."""
    X = np.atleast_2d(X)
    d = X.shape[1]
    mi = multi_indices(n, d)
    per_dim = [lagrange_1d(n, X[:, k]) for k in range(d)]
    out = np.ones((X.shape[0], mi.shape[0]))
    for k in range(d):
        out *= per_dim[k][:, mi[:, k]]
    return out


def node_grid(n: int, d: int) -> np.ndarray:
    """Reference coordinates (n^d, d) of the tensor nodes."""
    return nodes(n)[multi_indices(n, d)]
