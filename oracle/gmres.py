"""Right- and left-preconditioned GMRES (oracle; test infrastructure).

Sec. 3.2: non-restarted GMRES with a relative-residual tolerance on
||b - A x|| / ||b||, at most 500 iterations, with the IFMM as the right
preconditioner and the FMM product for A. App. B compares left and right
preconditioning; the right-preconditioned variant is the paper's default.

Reading: x0 = 0; the preconditioned directions Z_k = P^-1 v_k are stored
(flexible GMRES form), classical Gram-Schmidt with one re-orthogonalisation;
the stopping test uses the Arnoldi residual estimate and the true residual
is recomputed at exit.
"""
from __future__ import annotations

import numpy as np


def gmres_right(apply_A, apply_Minv, b, tol=1e-10, maxit=500):
    b = np.asarray(b, dtype=np.float64)
    n = b.shape[0]
    beta = float(np.linalg.norm(b))
    if beta == 0.0:
        return np.zeros(n), 0, 0.0, [0.0]
    V = np.zeros((n, maxit + 1))
    Z = np.zeros((n, maxit))
    H = np.zeros((maxit + 1, maxit))
    cs = np.zeros(maxit)
    sn = np.zeros(maxit)
    g = np.zeros(maxit + 1)
    g[0] = beta
    V[:, 0] = b / beta
    hist = [1.0]
    k = 0
    for k in range(maxit):
        Z[:, k] = apply_Minv(V[:, k])
        w = apply_A(Z[:, k])
        h = np.zeros(k + 2)
        for _ in range(2):                      # CGS2
            c = V[:, :k + 1].T @ w
            w = w - V[:, :k + 1] @ c
            h[:k + 1] += c
        h[k + 1] = np.linalg.norm(w)
        if h[k + 1] > 0:
            V[:, k + 1] = w / h[k + 1]
        # apply previous Givens rotations
        for j in range(k):
            t = cs[j] * h[j] + sn[j] * h[j + 1]
            h[j + 1] = -sn[j] * h[j] + cs[j] * h[j + 1]
            h[j] = t
        den = np.hypot(h[k], h[k + 1])
        cs[k] = h[k] / den if den > 0 else 1.0
        sn[k] = h[k + 1] / den if den > 0 else 0.0
        h[k] = den
        h[k + 1] = 0.0
        H[:k + 2, k] = h
        g[k + 1] = -sn[k] * g[k]
        g[k] = cs[k] * g[k]
        hist.append(abs(g[k + 1]) / beta)
        if abs(g[k + 1]) <= tol * beta:
            k += 1
            break
    else:
        k = maxit
    y = np.linalg.solve(np.triu(H[:k, :k]), g[:k]) if k > 0 else np.zeros(0)
    x = Z[:, :k] @ y
    res = float(np.linalg.norm(b - apply_A(x)) / beta)
    return x, k, res, hist


def gmres_left(apply_A, apply_Minv, b, tol=1e-10, maxit=500):
    """Left-preconditioned GMRES (App. B): the same non-restarted GMRES on the
    system P^-1 A x = P^-1 b, with P^-1 the IFMM preconditioner.

    The monitored residual is the preconditioned one,
    ||P^-1 (b - A x)|| / ||P^-1 b||, which is what the App. B tables report
    for the left variant. x0 = 0, classical Gram-Schmidt with one
    re-orthogonalisation, x = V_k y_k. Returns (x, iterations, preconditioned
    relative residual recomputed at exit, true relative residual
    ||b - A x|| / ||b||, history of the Arnoldi estimate).
    """
    b = np.asarray(b, dtype=np.float64)
    n = b.shape[0]
    r0 = np.asarray(apply_Minv(b), dtype=np.float64)
    beta = float(np.linalg.norm(r0))
    bnorm = float(np.linalg.norm(b))
    if beta == 0.0:
        return np.zeros(n), 0, 0.0, 0.0, [0.0]
    V = np.zeros((n, maxit + 1))
    H = np.zeros((maxit + 1, maxit))
    cs = np.zeros(maxit)
    sn = np.zeros(maxit)
    g = np.zeros(maxit + 1)
    g[0] = beta
    V[:, 0] = r0 / beta
    hist = [1.0]
    k = 0
    for k in range(maxit):
        w = apply_Minv(apply_A(V[:, k]))
        h = np.zeros(k + 2)
        for _ in range(2):                      # CGS2
            c = V[:, :k + 1].T @ w
            w = w - V[:, :k + 1] @ c
            h[:k + 1] += c
        h[k + 1] = np.linalg.norm(w)
        if h[k + 1] > 0:
            V[:, k + 1] = w / h[k + 1]
        for j in range(k):
            t = cs[j] * h[j] + sn[j] * h[j + 1]
            h[j + 1] = -sn[j] * h[j] + cs[j] * h[j + 1]
            h[j] = t
        den = np.hypot(h[k], h[k + 1])
        cs[k] = h[k] / den if den > 0 else 1.0
        sn[k] = h[k + 1] / den if den > 0 else 0.0
        h[k] = den
        h[k + 1] = 0.0
        H[:k + 2, k] = h
        g[k + 1] = -sn[k] * g[k]
        g[k] = cs[k] * g[k]
        hist.append(abs(g[k + 1]) / beta)
        if abs(g[k + 1]) <= tol * beta:
            k += 1
            break
    else:
        k = maxit
    y = np.linalg.solve(np.triu(H[:k, :k]), g[:k]) if k > 0 else np.zeros(0)
    x = V[:, :k] @ y
    r = b - apply_A(x)
    res_prec = float(np.linalg.norm(apply_Minv(r)) / beta)
    res_true = float(np.linalg.norm(r) / bnorm)
    return x, k, res_prec, res_true, hist
