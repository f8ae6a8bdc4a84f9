"""Brute-force quadrature used to pin the oracle's closed forms.

Tetrahedron: collapsed (Duffy) Gauss-Legendre product rule,
  l1 = u, l2 = v (1-u), l3 = w (1-u)(1-v),  Jacobian (1-u)^2 (1-v),
exact for polynomials of total degree <= 2n-3 with n points per direction.
Triangle: the same collapse in two variables.
"""
import numpy as np


def tet_rule(n=4):
    x, w = np.polynomial.legendre.leggauss(n)
    x = 0.5 * (x + 1.0); w = 0.5 * w
    U, V, W = np.meshgrid(x, x, x, indexing="ij")
    WU, WV, WW = np.meshgrid(w, w, w, indexing="ij")
    l1 = U; l2 = V * (1 - U); l3 = W * (1 - U) * (1 - V)
    l0 = 1 - l1 - l2 - l3
    wt = WU * WV * WW * (1 - U) ** 2 * (1 - V)
    lam = np.stack([l0.ravel(), l1.ravel(), l2.ravel(), l3.ravel()], axis=1)
    return lam, 6.0 * wt.ravel()        # weights sum to 1 (fraction of volume)


def tri_rule(n=5):
    x, w = np.polynomial.legendre.leggauss(n)
    x = 0.5 * (x + 1.0); w = 0.5 * w
    U, V = np.meshgrid(x, x, indexing="ij")
    WU, WV = np.meshgrid(w, w, indexing="ij")
    l1 = U; l2 = V * (1 - U); l0 = 1 - l1 - l2
    wt = WU * WV * (1 - U)
    lam = np.stack([l0.ravel(), l1.ravel(), l2.ravel()], axis=1)
    return lam, 2.0 * wt.ravel()        # weights sum to 1 (fraction of area)


def tet_volume(X):
    return abs(np.linalg.det(X[1:] - X[0])) / 6.0


def barycentric(X, pts):
    """Barycentric coordinates of pts in tetrahedron X by a 4x4 solve."""
    Mx = np.vstack([X.T, np.ones(4)])
    rhs = np.vstack([pts.T, np.ones(len(pts))])
    return np.linalg.solve(Mx, rhs).T


def bary_grads(X):
    """Barycentric gradients of tetrahedra X [...,4,3] from the inverse of
    the 4x4 affine matrix [[x^T], [1]]: lambda = inv @ [x; 1]."""
    X = np.asarray(X)
    M = np.concatenate([np.swapaxes(X, -1, -2), np.ones(X.shape[:-2] + (1, 4))], axis=-2)
    inv = np.linalg.inv(M)
    return inv[..., :, :3]


def whitney(X, pts, a, b):
    """Whitney edge function l_a grad l_b - l_b grad l_a at pts."""
    lam = barycentric(X, pts)
    g = bary_grads(X)
    return lam[:, a, None] * g[b][None, :] - lam[:, b, None] * g[a][None, :]


def curl_fd(fun, pts, h):
    """Curl of a vector field by central differences (exact for linear fields
    up to rounding)."""
    J = np.zeros((len(pts), 3, 3))
    for d in range(3):
        e = np.zeros(3); e[d] = h
        J[:, :, d] = (fun(pts + e) - fun(pts - e)) / (2 * h)
    return np.stack([J[:, 2, 1] - J[:, 1, 2], J[:, 0, 2] - J[:, 2, 0], J[:, 1, 0] - J[:, 0, 1]], axis=1)
