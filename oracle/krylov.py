"""Right-preconditioned flexible GMRES (the Krylov solver of Sec. IV-C).

TEST INFRASTRUCTURE ONLY (see the package docstring).

Each right-hand side is solved on its own (the GPU path runs them as one
pseudo-block).  Readings where the paper only says "GMRES": x0 = 0,
restart length m, classical Gram-Schmidt applied twice, complex Givens
rotations, Hermitian inner product, stop when the Arnoldi residual estimate
falls below rtol ||b|| and the true residual confirms it.  Flexible
(storing the preconditioned vectors) so that a nonlinear preconditioner is
allowed.  Iteration counts depend on rounding order: parity unpinned.
"""
from __future__ import annotations

import numpy as np


def givens(a: complex, b: complex):
    """(c, s) with [[c, s], [-conj(s), c]] [a; b] = [r; 0], c real."""
    if b == 0:
        return 1.0, 0.0
    if a == 0:
        return 0.0, np.conj(b) / abs(b)
    den = np.hypot(abs(a), abs(b))
    c = abs(a) / den
    s = (a / abs(a)) * np.conj(b) / den
    return c, s


def fgmres(A_mul, M_apply, b, rtol=1e-8, restart=40, maxit=2000, x0=None, callback=None):
    """Solve A x = b for one right-hand side.  Returns (x, iters, true relres, history)."""
    b = np.asarray(b, dtype=np.complex128)
    n = b.shape[0]
    x = np.zeros(n, dtype=np.complex128) if x0 is None else np.array(x0, dtype=np.complex128)
    bnorm = np.linalg.norm(b)
    if bnorm == 0:
        return x, 0, 0.0, []
    hist = []
    it = 0
    r = b - A_mul(x) if x0 is not None else b.copy()
    while True:
        beta = np.linalg.norm(r)
        if beta <= rtol * bnorm or it >= maxit:
            break
        m = restart
        V = np.zeros((m + 1, n), dtype=np.complex128)
        Z = np.zeros((m, n), dtype=np.complex128)
        H = np.zeros((m + 1, m), dtype=np.complex128)
        cs = np.zeros(m); sn = np.zeros(m, dtype=np.complex128)
        g = np.zeros(m + 1, dtype=np.complex128)
        g[0] = beta
        V[0] = r / beta
        k_done = 0
        for k in range(m):
            if callback is not None:
                callback(it, x, r, V[k], beta)
            Z[k] = M_apply(V[k])
            w = A_mul(Z[k])
            h = V[:k + 1].conj() @ w
            w = w - V[:k + 1].T @ h
            h2 = V[:k + 1].conj() @ w
            w = w - V[:k + 1].T @ h2
            h = h + h2
            hn = np.linalg.norm(w)
            H[:k + 1, k] = h
            H[k + 1, k] = hn
            if hn > 0:
                V[k + 1] = w / hn
            for j in range(k):
                t = cs[j] * H[j, k] + sn[j] * H[j + 1, k]
                H[j + 1, k] = -np.conj(sn[j]) * H[j, k] + cs[j] * H[j + 1, k]
                H[j, k] = t
            c, s = givens(H[k, k], H[k + 1, k])
            cs[k], sn[k] = c, s
            H[k, k] = c * H[k, k] + s * H[k + 1, k]
            H[k + 1, k] = 0.0
            g[k + 1] = -np.conj(s) * g[k]
            g[k] = c * g[k]
            it += 1
            k_done = k + 1
            hist.append(abs(g[k + 1]) / bnorm)
            if abs(g[k + 1]) <= rtol * bnorm or hn == 0 or it >= maxit:
                break
        y = np.zeros(k_done, dtype=np.complex128)
        for i in range(k_done - 1, -1, -1):
            y[i] = (g[i] - H[i, i + 1:k_done] @ y[i + 1:]) / H[i, i]
        x = x + Z[:k_done].T @ y
        r = b - A_mul(x)
    return x, it, np.linalg.norm(r) / bnorm, hist


def fgmres_block(A, M_apply, B, rtol=1e-8, restart=40, maxit=2000):
    """Independent FGMRES on every column of B."""
    X = np.zeros_like(B, dtype=np.complex128)
    its, res = [], []
    for j in range(B.shape[1]):
        x, it, rr, _ = fgmres(lambda v: A @ v, M_apply, B[:, j], rtol, restart, maxit)
        X[:, j] = x
        its.append(it); res.append(rr)
    return X, np.array(its), np.array(res)
