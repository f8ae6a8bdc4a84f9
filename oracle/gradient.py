"""Misfit, Tikhonov term and adjoint-state gradient of the inverse problem.

TEST INFRASTRUCTURE ONLY (see the package docstring).

Cost (Sec. IV-D, eq. (4)), with kappa = k^2 = k0^2 eps:

    J(eps) = 1/2 sum_ij w_ij |S_ij(eps) - S^meas_ij|^2 + alpha R,
    R      = 1/2 int |grad kappa|^2,

w_ij = 1 / |S^empty_ij|^2 supplied by the caller.  The permittivity is
piecewise linear, eps = sum_n eps_n lambda_n.  With S_ij = r_i^T u_j,
A u_j = b_j and A symmetric (no conjugation in eq. (2)), a perturbation of
eps gives dA = -k0^2 sum_n d eps_n M_n, M_n = sum_T M_{T,n}, and

    dJ = Re sum_n G_n d eps_n,   G_n = k0^2 sum_j lambda_j^T M_n u_j,
    A lambda_j = sum_i w_ij conj(d_ij) r_i          (adjoint, same matrix),

so dJ/dRe eps_n = Re G_n and dJ/dIm eps_n = -Im G_n; the complex gradient
g = dJ/dRe + j dJ/dIm is conj(G_n).  R = 1/2 k0^4 eps^H K1 eps with K1 the
P1 stiffness matrix adds alpha k0^4 (K1 eps)_n.  The outer boundary uses the
fixed background k_b, so it does not depend on eps.

Pinned by central finite differences of J (direct solves) and by K1 applied
to a linear field vanishing at interior vertices.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp

from . import fem


def p1_stiffness(topo: fem.Topology):
    """(K1)_nm = sum_T |T| grad l_n . grad l_m (real, [nv, nv])."""
    X = topo.xyz[topo.tet_sorted]
    g, vol = fem.barycentric_gradients(X)
    Ke = vol[:, None, None] * np.einsum("tid,tjd->tij", g, g)
    r = np.repeat(topo.tet_sorted, 4, axis=1).ravel()
    c = np.tile(topo.tet_sorted, (1, 4)).ravel()
    return sp.csr_matrix((Ke.ravel(), (r, c)), shape=(topo.nv, topo.nv))


def tikhonov(topo: fem.Topology, eps, freq_hz):
    """R = 1/2 int |grad kappa|^2 = 1/2 k0^4 Re(eps^H K1 eps), and K1 eps."""
    k0 = fem.k0_of(freq_hz)
    K1 = p1_stiffness(topo)
    Ke = K1 @ eps
    return 0.5 * k0 ** 4 * np.real(np.vdot(eps, Ke)), Ke


def misfit(topo: fem.Topology, eps, freq_hz, eps_b, pos, mom, S_meas, w):
    """J_misfit and the intermediate fields of the forward problem."""
    A = fem.assemble(topo, eps, 1, freq_hz, eps_b)
    R = fem.functionals(topo, pos, mom)
    B = -1j * fem.omega_mu0(freq_hz) * R
    U = fem.solve_direct(A, B)
    S = fem.scattering(R, U)
    d = S - S_meas
    return 0.5 * float(np.sum(w * np.abs(d) ** 2)), (A, R, U, S, d)


def cost(topo, eps, freq_hz, eps_b, pos, mom, S_meas, w, alpha):
    Jm, _ = misfit(topo, eps, freq_hz, eps_b, pos, mom, S_meas, w)
    Rv, _ = tikhonov(topo, eps, freq_hz)
    return Jm + alpha * Rv


def gradient(topo: fem.Topology, eps, freq_hz, eps_b, pos, mom, S_meas, w, alpha):
    """(J, g) with g_n = conj(G_n) + alpha k0^4 (K1 eps)_n (complex, [nv])."""
    eps = np.asarray(eps, dtype=np.complex128)
    k0 = fem.k0_of(freq_hz)
    Jm, (A, R, U, S, d) = misfit(topo, eps, freq_hz, eps_b, pos, mom, S_meas, w)
    Badj = R @ (w * np.conj(d))                      # [E, ntx]: sum_i w_ij conj(d_ij) r_i
    Lam = fem.solve_direct(A, Badj)
    X = topo.xyz[topo.tet_sorted]
    Mn = fem.element_mass_p1(X)                      # [T,4,6,6]
    lt = Lam[topo.t2e]                               # [T,6,ntx]
    ut = U[topo.t2e]
    W = np.einsum("tpj,tqj->tpq", lt, ut)            # sum over transmitters
    Gt = (k0 * k0) * np.einsum("tnpq,tpq->tn", Mn, W)
    G = np.zeros(topo.nv, dtype=np.complex128)
    np.add.at(G, topo.tet_sorted, Gt)
    Rv, Ke = tikhonov(topo, eps, freq_hz)
    g = np.conj(G) + alpha * k0 ** 4 * Ke
    return Jm + alpha * Rv, g, S
