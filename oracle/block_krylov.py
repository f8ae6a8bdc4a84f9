"""Block flexible GMRES: one Krylov space shared by all right-hand sides.

TEST INFRASTRUCTURE ONLY (see the package docstring).

The Krylov solver of Sec. IV-C is GMRES; with many transmitters per
permittivity (one per antenna) the right-hand sides form a block B, and the
block variant builds a single block Krylov space from the residual block
R0 = B - A X0 and minimises every column's residual over it. Readings where
the paper only says "GMRES", kept the same as the single-vector oracle:
X0 = 0, right preconditioning, flexible (the preconditioned blocks Z_k are
stored), restart after m block steps, classical block Gram-Schmidt applied
twice, stop when every column's Arnoldi residual estimate falls below
rtol ||b_j|| and the true residual confirms it.

Block Arnoldi (Saad, Iterative Methods for Sparse Linear Systems, 2nd ed.,
Sec. 6.12): R0 = V_0 S0 (QR); for k = 0, 1, ...: Z_k = M^{-1} V_k,
W = A Z_k, H_{i,k} = V_i^H W (twice, CGS2), W = V_{k+1} H_{k+1,k} (QR).
The block Hessenberg matrix Hbar_k ((k+2)s x (k+1)s) then satisfies
A [Z_0 .. Z_k] = [V_0 .. V_{k+1}] Hbar_k, and Y_k = argmin ||E S0 - Hbar_k Y||_F
(E: the first s columns of the identity) gives X = X0 + [Z_0 .. Z_k] Y_k;
column j's residual norm is the norm of column j of E S0 - Hbar_k Y_k.
QR factorisations and the small least-squares problems use numpy.
A residual block or new block of lower numerical rank than s (relative
threshold 1e-12 on the diagonal of its R factor) ends the cycle (after the
first step) or raises (at the start of a cycle).
"""
from __future__ import annotations

import numpy as np


class RankDeficient(RuntimeError):
    pass


def _qr_full_rank(W, tol=1e-12):
    Q, R = np.linalg.qr(W)
    d = np.abs(np.diag(R))
    ok = d.size == 0 or d.min() > tol * max(d.max(), 1e-300)
    return Q, R, ok


def block_fgmres(A_mul, M_apply, B, rtol=1e-8, restart=30, maxit=2000, history=False):
    """Solve A X = B (B [n, s]). Returns (X, block steps, true relres per
    column, per-step max relative residual estimates)."""
    B = np.asarray(B, dtype=np.complex128)
    n, s = B.shape
    X = np.zeros_like(B)
    bn = np.linalg.norm(B, axis=0)
    if np.any(bn == 0):
        raise RankDeficient("zero right-hand side column")
    steps = 0
    hist = []
    R = B.copy()
    while True:
        rel = np.linalg.norm(R, axis=0) / bn
        if rel.max() <= rtol or steps >= maxit:
            break
        V0, S0, ok = _qr_full_rank(R)
        if not ok:
            raise RankDeficient("residual block of lower rank than the number of right-hand sides")
        m = restart
        V = [V0]
        Z = []
        H = np.zeros(((m + 1) * s, m * s), dtype=np.complex128)
        G = np.zeros(((m + 1) * s, s), dtype=np.complex128)
        G[:s] = S0
        Y = None
        kk = 0
        for k in range(m):
            Zk = M_apply(V[k])
            W = A_mul(Zk)
            Vk = np.hstack(V)                          # [n, (k+1)s]
            h = Vk.conj().T @ W
            W = W - Vk @ h
            h2 = Vk.conj().T @ W
            W = W - Vk @ h2
            Q, Rk, ok = _qr_full_rank(W)
            if not ok and k > 0:
                break                                   # this step is not used
            Z.append(Zk)
            H[:(k + 1) * s, k * s:(k + 1) * s] = h + h2
            H[(k + 1) * s:(k + 2) * s, k * s:(k + 1) * s] = Rk
            V.append(Q)
            steps += 1
            kk = k + 1
            Hk = H[:(k + 2) * s, :(k + 1) * s]
            Y = np.linalg.lstsq(Hk, G[:(k + 2) * s], rcond=None)[0]
            est = np.linalg.norm(G[:(k + 2) * s] - Hk @ Y, axis=0) / bn
            hist.append(float(est.max()))
            if est.max() <= rtol or steps >= maxit:
                break
        if kk == 0:
            raise RankDeficient("first block of the cycle lost rank")
        X = X + np.hstack(Z[:kk]) @ Y
        R = B - A_mul(X)
    rel = np.linalg.norm(R, axis=0) / bn
    return X, steps, rel, hist
