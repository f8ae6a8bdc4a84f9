"""Waveguide ports and metallic walls (TEST INFRASTRUCTURE ONLY).

Boundary conditions of eq. (1) in their port form (Sec. IV-B): metallic
walls Gamma_m (n x E = 0), transmitting/receiving waveguide ports where the
dominant TE10 mode is imposed through (curl E) x n + j beta n x (E x n) = g,
g = 2 j beta E^TE10, and the scattering coefficients of eq. (3).

A port is a planar rectangle (centre c, outward normal n, broad-side unit
vector u, width a along u, height b along v = n x u) filled near the port
with permittivity eps; its TE10 profile is e(x) = sin(pi (s + a/2) / a) v,
s = (x - c).u, and its propagation constant beta = sqrt(k0^2 eps - (pi/a)^2)
on the branch with Im beta <= 0 (waves e^{-j beta z} that decay, e^{jwt}).

* A boundary face belongs to port p when its centroid lies in the port's
  plane and rectangle (relative tolerance 1e-6 of the port size).
* Port faces carry j beta_p B_F (the impedance face matrix with k -> beta_p);
  the other boundary faces are metallic (pec=True) or keep the impedance
  condition with k_b of eps_b (pec=False).
* Metallic edges (every edge of a non-port boundary face when pec=True) are
  eliminated symmetrically: their rows and columns are cleared and the
  diagonal set to 1, with zero right-hand side.
* Port p as transmitter: b_e = int_{Gamma_p} g_p . N_e dS; as receiver:
  r_e = int_{Gamma_p} e_p . N_e dS / int_{Gamma_p} e_p . e_p dS, and
  S = R^T U - I (the incident wave of unit amplitude removed on the
  transmitting port).
Surface integrals use a 7-point degree-5 triangle rule.

Pinned by the straight-waveguide closed form (S21 = e^{-j beta L}, S11 = 0
for the exact mode), reciprocity and, for a lossless medium, power balance.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np
import scipy.sparse as sp

from oracle import fem


@dataclass
class Port:
    centre: tuple
    normal: tuple
    u: tuple
    a: float
    b: float
    eps: complex


def _frame(p: Port):
    n = np.asarray(p.normal, float)
    n = n / np.linalg.norm(n)
    u = np.asarray(p.u, float)
    u = u - (u @ n) * n
    u = u / np.linalg.norm(u)
    v = np.cross(n, u)
    return np.asarray(p.centre, float), n, u, v


def beta(k0: float, p: Port) -> complex:
    b = np.sqrt(complex(k0 * k0 * p.eps - (np.pi / p.a) ** 2))
    return -b if b.imag > 0 else b


def mode(p: Port, x):
    """TE10 profile e(x) [..., 3] (real)."""
    c, n, u, v = _frame(p)
    s = (x - c) @ u
    return np.sin(np.pi * (s + 0.5 * p.a) / p.a)[..., None] * v


def classify(topo: fem.Topology, ports):
    """Port index of every boundary face (-1: not on a port)."""
    P = topo.xyz[topo.bface_verts]
    cen = P.mean(axis=1)
    out = np.full(len(cen), -1, dtype=np.int64)
    for i, p in enumerate(ports):
        c, n, u, v = _frame(p)
        tol = 1e-6 * (p.a + p.b)
        d = cen - c
        on = (np.abs(d @ n) <= tol) & (np.abs(d @ u) <= 0.5 * p.a + tol) & (np.abs(d @ v) <= 0.5 * p.b + tol)
        out[on & (out < 0)] = i
    return out


def pec_edges(topo: fem.Topology, face_port, pec: bool):
    if not pec:
        return np.zeros(0, dtype=np.int64)
    return np.unique(topo.bface_edges[face_port < 0].ravel())


def assemble(topo: fem.Topology, eps, eps_kind: int, freq_hz: float, eps_b: complex, ports, pec: bool = True):
    """A with port faces, metallic or impedance walls, metallic edges
    eliminated; returns (A, face_port, pec edge ids)."""
    k0 = fem.k0_of(freq_hz)
    fp = classify(topo, ports)
    Ae = fem.element_operator(topo, eps, eps_kind, k0)
    P = topo.xyz[topo.bface_verts]
    Bf = fem.face_matrix(P)
    kf = np.zeros(len(fp), dtype=np.complex128)
    for i, p in enumerate(ports):
        kf[fp == i] = beta(k0, p)
    if not pec:
        kf[fp < 0] = fem.wavenumber(k0, eps_b)
    Bf = 1j * kf[:, None, None] * Bf
    r1 = np.repeat(topo.t2e, 6, axis=1).ravel()
    c1 = np.tile(topo.t2e, (1, 6)).ravel()
    r2 = np.repeat(topo.bface_edges, 3, axis=1).ravel()
    c2 = np.tile(topo.bface_edges, (1, 3)).ravel()
    data = fem._deterministic_csr(topo, np.r_[r1, r2], np.r_[c1, c2], np.r_[Ae.reshape(-1), Bf.reshape(-1)])
    A = sp.csr_matrix((data, topo.col, topo.row_ptr), shape=(topo.ne, topo.ne))
    pe = pec_edges(topo, fp, pec)
    if len(pe):
        keep = np.ones(topo.ne)
        keep[pe] = 0.0
        A = sp.diags(keep) @ A @ sp.diags(keep) + sp.diags(1.0 - keep)
    return A.tocsr(), fp, pe


# 7-point degree-5 rule on the reference triangle (barycentric, weights sum 1)
_A1, _B1 = 0.059715871789770, 0.470142064105115
_A2, _B2 = 0.797426985353087, 0.101286507323456
_TRI = np.array([[1 / 3, 1 / 3, 1 / 3], [_A1, _B1, _B1], [_B1, _A1, _B1], [_B1, _B1, _A1],
                 [_A2, _B2, _B2], [_B2, _A2, _B2], [_B2, _B2, _A2]])
_TRW = np.array([0.225] + [0.132394152788506] * 3 + [0.125939180544827] * 3)


def _face_quadrature(topo, faces):
    """Points [F,7,3], weights*area [F,7], 2-D Whitney values [F,7,3(edges),3]."""
    P = topo.xyz[topo.bface_verts[faces]]                       # [F,3,3]
    g, area = fem.surface_gradients(P)                          # [F,3,3], [F]
    pts = np.einsum("qi,fid->fqd", _TRI, P)
    N = np.empty((len(faces), len(_TRW), 3, 3))
    for k, (a, b) in enumerate(fem.FACE_EDGES):
        la = _TRI[:, a][None, :, None]
        lb = _TRI[:, b][None, :, None]
        N[:, :, k, :] = la * g[:, None, b, :] - lb * g[:, None, a, :]
    return pts, _TRW[None, :] * area[:, None], N


def _port_integrals(topo, ports, face_port, values):
    """Columns p: int_{Gamma_p} values(p, x) . N_e dS."""
    out = np.zeros((topo.ne, len(ports)), dtype=np.complex128)
    for i, p in enumerate(ports):
        faces = np.nonzero(face_port == i)[0]
        if len(faces) == 0:
            continue
        pts, w, N = _face_quadrature(topo, faces)
        f = values(i, p, pts)                                   # [F,7,3]
        contrib = np.einsum("fq,fqd,fqkd->fk", w, f, N)         # [F,3]
        np.add.at(out[:, i], topo.bface_edges[faces].ravel(), contrib.ravel())
    return out


def port_rhs(topo, ports, face_port, pec_e, freq_hz: float):
    k0 = fem.k0_of(freq_hz)
    B = _port_integrals(topo, ports, face_port, lambda i, p, x: 2j * beta(k0, p) * mode(p, x))
    B[pec_e] = 0.0
    return B


def port_functionals(topo, ports, face_port, pec_e):
    R = _port_integrals(topo, ports, face_port, lambda i, p, x: mode(p, x))
    for i, p in enumerate(ports):
        faces = np.nonzero(face_port == i)[0]
        pts, w, _ = _face_quadrature(topo, faces)
        e = mode(p, pts)
        R[:, i] /= np.einsum("fq,fqd,fqd->", w, e, e)
    R[pec_e] = 0.0
    return R


def scattering(R, U):
    return R.T @ U - np.eye(R.shape[1], U.shape[1])


def waveguide(a: float, b: float, length: float, n: tuple, eps: complex):
    """Straight rectangular waveguide [0,a]x[0,b]x[0,L] (Kuhn lattice with
    n = (na, nb, nL) cells), port 0 at z = 0 (normal -z), port 1 at z = L."""
    import workload
    xyz, tet = workload.kuhn_box(n, (0.0, 0.0, 0.0), (a, b, length))
    # u flips with n so that both ports see the same field direction v
    ports = [Port((a / 2, b / 2, 0.0), (0, 0, -1), (1, 0, 0), a, b, eps),
             Port((a / 2, b / 2, length), (0, 0, 1), (-1, 0, 0), a, b, eps)]
    return xyz, tet, ports
