"""Lowest-order Nedelec discretisation of the time-harmonic Maxwell problem.

TEST INFRASTRUCTURE ONLY (see the package docstring).

Problem (paper Sec. IV-B, eq. (1) and its weak form (2)): find E in
H(curl) with

    int curl E . curl v - k^2 E . v  +  int_{dOmega} j k (E x n).(v x n)
        = -j omega mu0 int J . v ,

k^2 = k0^2 eps_r, exp(+j omega t).  The outer boundary carries the
first-order impedance (absorbing) condition of the open sides; the source is
a point dipole J = p delta(x - x_s) instead of the waveguide port.  The
discrete space is the first-order Nedelec (edge) element on tetrahedra
(Sec. IV-D: r = 1).  No conjugation appears in (2), so the matrix is
complex symmetric.
"""
from __future__ import annotations

import math

import numpy as np
import scipy.linalg as sla
import scipy.sparse as sp
import scipy.sparse.linalg as spla

EPS0 = 8.8541878128e-12
MU0 = 4.0e-7 * math.pi
C0 = 299792458.0

# local edges of a tetrahedron whose vertices are sorted by global id; the
# orientation low -> high id is therefore the global edge orientation.
LOCAL_EDGES = ((0, 1), (0, 2), (0, 3), (1, 2), (1, 3), (2, 3))
# local faces, each a sorted vertex triple, and the local edges on it
LOCAL_FACES = ((0, 1, 2), (0, 1, 3), (0, 2, 3), (1, 2, 3))
FACE_EDGES = ((0, 1), (0, 2), (1, 2))       # edges of a sorted triangle


def k0_of(freq_hz: float) -> float:
    return 2.0 * math.pi * freq_hz / C0


def omega_mu0(freq_hz: float) -> float:
    return 2.0 * math.pi * freq_hz * MU0


def wavenumber(k0: float, eps: complex) -> complex:
    """k = k0 sqrt(eps_r), principal branch (Re k > 0, Im k <= 0 for lossy eps)."""
    return k0 * np.sqrt(np.complex128(eps))


# --------------------------------------------------------------------------
# O1: topology
# --------------------------------------------------------------------------

class Topology:
    """Edges, tetrahedron->edge map, boundary faces and the CSR pattern.

    Definitions (pinned by the closed-form Kuhn counts and Euler's formula):
      * each tetrahedron's vertices are sorted by id;
      * global edges are the distinct (vmin, vmax) pairs, numbered in
        lexicographic order;
      * boundary faces are the sorted vertex triples that belong to exactly
        one tetrahedron, numbered in lexicographic order;
      * the matrix pattern holds (e, f) whenever edges e and f share a
        tetrahedron; columns sorted within a row.
    """

    def __init__(self, xyz, tet):
        xyz = np.asarray(xyz, dtype=np.float64)
        tet = np.asarray(tet, dtype=np.int64)
        self.xyz = xyz
        self.tet_in = tet
        self.nv = xyz.shape[0]
        self.nt = tet.shape[0]
        ts = np.sort(tet, axis=1)
        self.tet_sorted = ts
        nv = np.int64(self.nv)
        a = ts[:, [e[0] for e in LOCAL_EDGES]]
        b = ts[:, [e[1] for e in LOCAL_EDGES]]
        keys = a * nv + b
        uniq, inv = np.unique(keys.ravel(), return_inverse=True)
        self.edges = np.stack([uniq // nv, uniq % nv], axis=1)
        self.ne = self.edges.shape[0]
        self.t2e = inv.reshape(self.nt, 6)
        # faces
        fk = []
        for f in LOCAL_FACES:
            fk.append((ts[:, f[0]] * nv + ts[:, f[1]]) * nv + ts[:, f[2]])
        fk = np.stack(fk, axis=1).ravel()
        ufk, finv, fcnt = np.unique(fk, return_inverse=True, return_counts=True)
        self.nfaces_total = ufk.shape[0]
        bmask = fcnt == 1
        occ = np.nonzero(bmask[finv])[0]          # flat (tet*4 + local face)
        order = np.argsort(fk[occ], kind="stable")
        occ = occ[order]
        self.bface_tet = occ // 4
        self.bface_local = occ % 4
        lf = np.array(LOCAL_FACES)
        self.bface_verts = ts[self.bface_tet[:, None], lf[self.bface_local]]
        le = {e: i for i, e in enumerate(LOCAL_EDGES)}
        fe = np.array([[le[(f[p], f[q])] for (p, q) in FACE_EDGES] for f in LOCAL_FACES])
        self.bface_edges = self.t2e[self.bface_tet[:, None], fe[self.bface_local]]
        # face id of every (tet, local face), and the second tet of interior faces
        self.face_of = finv.reshape(self.nt, 4)
        # CSR pattern
        rows = np.repeat(self.t2e, 6, axis=1).ravel()
        cols = np.tile(self.t2e, (1, 6)).ravel()
        pk = np.unique(rows * np.int64(self.ne) + cols)
        self.row_ptr = np.zeros(self.ne + 1, dtype=np.int64)
        np.add.at(self.row_ptr, pk // self.ne + 1, 1)
        self.row_ptr = np.cumsum(self.row_ptr)
        self.col = (pk % self.ne).astype(np.int64)
        self.nnz = self.col.shape[0]


# --------------------------------------------------------------------------
# O2/O3: basis and element matrices
# --------------------------------------------------------------------------

def barycentric_gradients(X):
    """X [...,4,3] vertex coordinates -> (grad lambda [...,4,3], volume [...]).

    lambda_1..3 are the coordinates s of x = x0 + sum_k s_k (x_k - x0);
    lambda_0 = 1 - sum.  With D the matrix whose rows are x_k - x0 the
    gradients of s_k are the rows of D^{-T}.
    """
    D = X[..., 1:, :] - X[..., :1, :]
    Dinv = np.linalg.inv(D)
    g = np.empty(X.shape, dtype=np.float64)
    g[..., 1:, :] = np.swapaxes(Dinv, -1, -2)
    g[..., 0, :] = -g[..., 1:, :].sum(axis=-2)
    vol = np.abs(np.linalg.det(D)) / 6.0
    return g, vol


def element_matrices(X):
    """Curl-curl K_T and mass M_T (6x6, local edge order LOCAL_EDGES).

    N_ab = l_a grad l_b - l_b grad l_a,  curl N_ab = 2 grad l_a x grad l_b,
    int_T l_i l_j = |T| (1 + delta_ij) / 20.
    Only the upper triangle is evaluated and mirrored so K_T, M_T are exactly
    symmetric.  Pinned by brute-force quadrature, the edge-moment property,
    K_T G_T = 0 and rank/definiteness checks.
    """
    g, vol = barycentric_gradients(X)
    nT = X.shape[:-2]
    K = np.zeros(nT + (6, 6))
    M = np.zeros(nT + (6, 6))
    G = np.einsum("...id,...jd->...ij", g, g)          # grad l_i . grad l_j
    curls = [2.0 * np.cross(g[..., a, :], g[..., b, :]) for (a, b) in LOCAL_EDGES]
    for p, (a, b) in enumerate(LOCAL_EDGES):
        for q in range(p, 6):
            c, d = LOCAL_EDGES[q]
            K[..., p, q] = vol * (curls[p] * curls[q]).sum(axis=-1)
            m = ((1 + (a == c)) * G[..., b, d] - (1 + (a == d)) * G[..., b, c]
                 - (1 + (b == c)) * G[..., a, d] + (1 + (b == d)) * G[..., a, c])
            M[..., p, q] = vol / 20.0 * m
            if q != p:
                K[..., q, p] = K[..., p, q]
                M[..., q, p] = M[..., p, q]
    return K, M


def _int_lll(n, i, j):
    """int_T l_n l_i l_j / |T|  =  3! alpha! / (|alpha|+3)!."""
    idx = [n, i, j]
    pw = [idx.count(k) for k in range(4)]
    num = 6 * math.prod(math.factorial(p) for p in pw)
    return num / math.factorial(6)


def element_mass_p1(X):
    """M_{T,n}[e,f] = int_T l_n N_e . N_f for n = 0..3 -> [...,4,6,6].

    Used for a piecewise-linear permittivity eps = sum_n eps_n l_n.
    Pinned by sum_n M_{T,n} = M_T and brute-force quadrature.
    """
    g, vol = barycentric_gradients(X)
    nT = X.shape[:-2]
    G = np.einsum("...id,...jd->...ij", g, g)
    out = np.zeros(nT + (4, 6, 6))
    for n in range(4):
        for p, (a, b) in enumerate(LOCAL_EDGES):
            for q in range(p, 6):
                c, d = LOCAL_EDGES[q]
                m = (_int_lll(n, a, c) * G[..., b, d] - _int_lll(n, a, d) * G[..., b, c]
                     - _int_lll(n, b, c) * G[..., a, d] + _int_lll(n, b, d) * G[..., a, c])
                out[..., n, p, q] = vol * m
                if q != p:
                    out[..., n, q, p] = out[..., n, p, q]
    return out


def surface_gradients(P):
    """P [...,3,3] triangle vertices -> (tangential grad of the 2-D
    barycentrics [...,3,3], area [...]).  With e1 = P1-P0, e2 = P2-P0 and the
    metric G = [e_i . e_j], grad l_{1,2} = G^{-1} rows combined with (e1, e2)."""
    e1 = P[..., 1, :] - P[..., 0, :]
    e2 = P[..., 2, :] - P[..., 0, :]
    g11 = (e1 * e1).sum(-1); g12 = (e1 * e2).sum(-1); g22 = (e2 * e2).sum(-1)
    det = g11 * g22 - g12 * g12
    i11 = g22 / det; i12 = -g12 / det; i22 = g11 / det
    gr = np.empty(P.shape)
    gr[..., 1, :] = i11[..., None] * e1 + i12[..., None] * e2
    gr[..., 2, :] = i12[..., None] * e1 + i22[..., None] * e2
    gr[..., 0, :] = -gr[..., 1, :] - gr[..., 2, :]
    area = 0.5 * np.sqrt(det)
    return gr, area


def face_matrix(P):
    """B_F[e,f] = int_F (N_e x n).(N_f x n) over the 3 edges of a triangle
    (vertices sorted by id, edge order FACE_EDGES); int_F l_i l_j =
    |F| (1 + delta_ij) / 12.  Tangential traces of the tetrahedral Nedelec
    functions are the 2-D Nedelec functions of the face."""
    g, area = surface_gradients(P)
    G = np.einsum("...id,...jd->...ij", g, g)
    B = np.zeros(P.shape[:-2] + (3, 3))
    for p, (a, b) in enumerate(FACE_EDGES):
        for q in range(p, 3):
            c, d = FACE_EDGES[q]
            m = ((1 + (a == c)) * G[..., b, d] - (1 + (a == d)) * G[..., b, c]
                 - (1 + (b == c)) * G[..., a, d] + (1 + (b == d)) * G[..., a, c])
            B[..., p, q] = area / 12.0 * m
            if q != p:
                B[..., q, p] = B[..., p, q]
    return B


# --------------------------------------------------------------------------
# O4: the global operator
# --------------------------------------------------------------------------

def tet_eps(topo: Topology, eps, eps_kind: int):
    """Per-tetrahedron permittivity: P0 value, or the vertex mean for P1."""
    eps = np.asarray(eps, dtype=np.complex128)
    if eps_kind == 0:
        return eps
    return eps[topo.tet_sorted].mean(axis=1)


def element_operator(topo: Topology, eps, eps_kind: int, k0: float):
    """Per-tetrahedron 6x6 blocks of K_T - k0^2 (eps M)_T (eq. (2), volume part)."""
    X = topo.xyz[topo.tet_sorted]
    K, M = element_matrices(X)
    eps = np.asarray(eps, dtype=np.complex128)
    if eps_kind == 0:
        return K - (k0 * k0) * eps[:, None, None] * M
    Mn = element_mass_p1(X)
    epsv = eps[topo.tet_sorted]                             # [T,4]
    Me = np.einsum("tn,tnij->tij", epsv, Mn)
    return K - (k0 * k0) * Me


def boundary_face_blocks(topo: Topology, kb: complex):
    """Per boundary face 3x3 blocks j k_b B_F (eq. (2), impedance part)."""
    P = topo.xyz[topo.bface_verts]
    return 1j * kb * face_matrix(P)


def _deterministic_csr(topo: Topology, rows, cols, vals):
    """Sum (row, col, val) triplets into the CSR pattern of topo, in the order
    the triplets are given (so equal triplet sequences give equal sums)."""
    key = rows.astype(np.int64) * topo.ne + cols
    rp = topo.row_ptr
    pat = np.repeat(np.arange(topo.ne, dtype=np.int64), np.diff(rp)) * topo.ne + topo.col
    pos = np.searchsorted(pat, key)
    assert np.all(pat[pos] == key)
    order = np.argsort(pos, kind="stable")
    pos_s = pos[order]
    vals_s = vals[order]
    start = np.r_[0, np.nonzero(np.diff(pos_s))[0] + 1]
    rank = np.arange(pos_s.shape[0]) - np.repeat(start, np.diff(np.r_[start, pos_s.shape[0]]))
    out = np.zeros(topo.nnz, dtype=vals.dtype)
    for r in range(int(rank.max()) + 1):
        m = rank == r
        out[pos_s[m]] += vals_s[m]
    return out


def assemble(topo: Topology, eps, eps_kind: int, freq_hz: float, eps_b: complex):
    """A = sum_T (K_T - k0^2 eps M_T) + j k_b sum_F B_F as CSR (scipy).

    Contributions to each entry are summed tetrahedra first (ascending id),
    then boundary faces (ascending id); A == A^T bitwise.  Pinned by the
    plane-wave convergence test, the curl kernel and symmetry.
    """
    k0 = k0_of(freq_hz)
    kb = wavenumber(k0, eps_b)
    Ae = element_operator(topo, eps, eps_kind, k0)
    Bf = boundary_face_blocks(topo, kb)
    r1 = np.repeat(topo.t2e, 6, axis=1).ravel()
    c1 = np.tile(topo.t2e, (1, 6)).ravel()
    r2 = np.repeat(topo.bface_edges, 3, axis=1).ravel()
    c2 = np.tile(topo.bface_edges, (1, 3)).ravel()
    rows = np.r_[r1, r2]; cols = np.r_[c1, c2]
    vals = np.r_[Ae.reshape(-1), Bf.reshape(-1)]
    data = _deterministic_csr(topo, rows, cols, vals)
    return sp.csr_matrix((data, topo.col, topo.row_ptr), shape=(topo.ne, topo.ne))


def curl_curl_matrix(topo: Topology):
    """K alone (k0 = 0, no boundary term) for the curl-kernel check."""
    X = topo.xyz[topo.tet_sorted]
    K, _ = element_matrices(X)
    r = np.repeat(topo.t2e, 6, axis=1).ravel()
    c = np.tile(topo.t2e, (1, 6)).ravel()
    return sp.csr_matrix((K.reshape(-1), (r, c)), shape=(topo.ne, topo.ne))


def gradient_matrix(topo: Topology):
    """Discrete gradient G [E,V]: (G phi)_e = phi_b - phi_a for edge a->b."""
    e = np.arange(topo.ne)
    r = np.r_[e, e]
    c = np.r_[topo.edges[:, 1], topo.edges[:, 0]]
    v = np.r_[np.ones(topo.ne), -np.ones(topo.ne)]
    return sp.csr_matrix((v, (r, c)), shape=(topo.ne, topo.nv))


# --------------------------------------------------------------------------
# O5: sources and receivers
# --------------------------------------------------------------------------

def locate(topo: Topology, x, tol: float = 1e-12):
    """All tetrahedra whose closure contains x: min barycentric >= -tol.
    Returns (tet ids ascending, barycentric gradients, barycentrics)."""
    X = topo.xyz[topo.tet_sorted]
    g, _ = barycentric_gradients(X)
    lam = np.einsum("tkd,td->tk", g, np.asarray(x)[None, :] - X[:, 0, :])
    lam[:, 0] += 1.0
    hit = np.nonzero(lam.min(axis=1) >= -tol)[0]
    return hit, g[hit], lam[hit]


def point_functional(topo: Topology, x, p):
    """r[e] = p . N_e(x) as a dense vector; for x on a shared face, edge or
    vertex the value is the mean over all tetrahedra containing x.
    Pinned by exact reproduction of constant fields (p . E0)."""
    hit, g, lam = locate(topo, x)
    if hit.size == 0:
        raise ValueError(f"point {x} lies outside the mesh")
    r = np.zeros(topo.ne, dtype=np.complex128)
    for t in range(hit.size):
        for le, (a, b) in enumerate(LOCAL_EDGES):
            N = lam[t, a] * g[t, b] - lam[t, b] * g[t, a]
            r[topo.t2e[hit[t], le]] += np.dot(np.asarray(p, dtype=np.complex128), N)
    return r / hit.size


def functionals(topo: Topology, pos, mom):
    """R [E, n] with column j = p_j . N_e(x_j)."""
    return np.stack([point_functional(topo, pos[j], mom[j]) for j in range(len(pos))], axis=1)


def dipole_rhs(topo: Topology, pos, mom, freq_hz: float):
    """b_j = -j omega mu0 p_j . N_e(x_j)  (right side of eq. (2) for J = p delta)."""
    return -1j * omega_mu0(freq_hz) * functionals(topo, pos, mom)


# --------------------------------------------------------------------------
# O6: direct solve
# --------------------------------------------------------------------------

def solve_direct(A, B, dense_max: int = 12000):
    """Exact solve A X = B: LAPACK dense LU (getrf/getrs) up to dense_max
    unknowns, sparse LU (SuperLU) beyond."""
    B = np.asarray(B)
    if A.shape[0] <= dense_max:
        lu = sla.lu_factor(A.toarray())
        return sla.lu_solve(lu, B)
    return sparse_lu(A).solve(np.asarray(B, dtype=np.complex128))


def sparse_lu(A):
    """SuperLU with minimum-degree ordering of A^T + A (the pattern is symmetric)."""
    return spla.splu(sp.csc_matrix(A), permc_spec="MMD_AT_PLUS_A",
                     options=dict(SymmetricMode=True))


def scattering(R_rx, U):
    """S = R_rx^T U (receiver responses of every transmitter)."""
    return R_rx.T @ U


# --------------------------------------------------------------------------
# helpers used by the plane-wave pin
# --------------------------------------------------------------------------

def edge_interpolant(topo: Topology, field, nq: int = 4):
    """u_e = int_e E . t ds (t from low to high id) by Gauss-Legendre."""
    xq, wq = np.polynomial.legendre.leggauss(nq)
    s = 0.5 * (xq + 1.0); w = 0.5 * wq
    xa = topo.xyz[topo.edges[:, 0]]; xb = topo.xyz[topo.edges[:, 1]]
    u = np.zeros(topo.ne, dtype=np.complex128)
    for sk, wk in zip(s, w):
        pts = xa + sk * (xb - xa)
        u += wk * (field(pts) * (xb - xa)).sum(axis=1)
    return u
