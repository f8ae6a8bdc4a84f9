"""Overlapping Schwarz pieces: partition, overlap, partition of unity,
colouring and the ORAS subdomain matrices.

TEST INFRASTRUCTURE ONLY (see the package docstring).

The paper (Sec. IV-C) solves each linear system with GMRES preconditioned
by Optimized Restricted Additive Schwarz: the mesh is split into overlapping
subdomains small enough for direct solvers, each subdomain problem carries
an impedance (transmission) condition on its artificial boundary, and the
local solutions are glued with a partition of unity:

    M^{-1} = sum_i R_i^T D_i B_i^{-1} R_i .

The paper does not say how the partition, the overlap or the partition of
unity are built; the readings used here are:
  * recursive coordinate bisection of tetrahedron centroids;
  * delta layers of vertex-adjacent tetrahedra of overlap;
  * integer vertex weights omega_i(v) = delta - (first layer of v), edge
    weight w_i(e) = omega_i(a) + omega_i(b), D_i = w_i / sum_j w_j;
  * B_i assembled from the tetrahedra of the overlapping subdomain, plus
    j k_T B_F on faces shared with an outside tetrahedron (k_T of the inside
    tetrahedron) and j k_b B_F on faces of the outer boundary.
"""
from __future__ import annotations

import numpy as np
import scipy.linalg as sla
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from . import fem


def tet_centroids_exact(xyz, tet):
    """Centroid ((x0 + x1) + x2) + x3, times 0.25, in input vertex order."""
    X = xyz[tet]
    return (((X[:, 0] + X[:, 1]) + X[:, 2]) + X[:, 3]) * 0.25


def rcb(xyz, tet, nsub: int):
    """Recursive coordinate bisection into nsub = 2^L parts.

    Each set is split along the axis of largest centroid extent (first axis
    on ties), ordered by (coordinate, tetrahedron id); the first floor(m/2)
    tetrahedra form the left part, which takes the lower half of the part
    numbers.  Pinned at the cube mesh by the 2x2x2 box split.
    """
    if nsub < 1 or nsub & (nsub - 1):
        raise ValueError("nsub must be a power of two")
    cen = tet_centroids_exact(np.asarray(xyz, np.float64), np.asarray(tet))
    part = np.empty(len(tet), dtype=np.int64)

    def split(ids, p0, np_):
        if np_ == 1:
            part[ids] = p0
            return
        c = cen[ids]
        ext = c.max(axis=0) - c.min(axis=0)
        ax = int(np.argmax(ext))
        order = np.lexsort((ids, c[:, ax]))
        m = ids.shape[0]
        split(ids[order[: m // 2]], p0, np_ // 2)
        split(ids[order[m // 2:]], p0 + np_ // 2, np_ // 2)

    split(np.arange(len(tet), dtype=np.int64), 0, nsub)
    return part


class Decomposition:
    """Overlapping subdomains, DOF lists, partition-of-unity weights, colours."""

    def __init__(self, topo: fem.Topology, nsub: int, overlap: int):
        if overlap < 1:
            raise ValueError("overlap must be >= 1 (the partition of unity needs it)")
        self.topo = topo
        self.nsub = nsub
        self.overlap = overlap
        self.part = rcb(topo.xyz, topo.tet_in, nsub)
        ts = topo.tet_sorted
        nt, nv = topo.nt, topo.nv
        v2t = sp.csr_matrix((np.ones(4 * nt, dtype=np.int8),
                             (ts.ravel(), np.repeat(np.arange(nt), 4))), shape=(nv, nt))
        self.tets, self.dofs, self.w, self.vlayer = [], [], [], []
        for i in range(nsub):
            inT = self.part == i
            layer = np.full(nv, -1, dtype=np.int64)
            layer[np.unique(ts[inT])] = 0
            for l in range(1, overlap + 1):
                touched = np.asarray(v2t[layer >= 0].sum(axis=0)).ravel() > 0
                inT = inT | touched
                vs = np.unique(ts[inT])
                new = vs[layer[vs] < 0]
                layer[new] = l
            tets_i = np.nonzero(inT)[0]
            dofs_i = np.unique(topo.t2e[tets_i])
            om = np.maximum(overlap - layer, 0)
            om[layer < 0] = 0
            ea, eb = topo.edges[dofs_i, 0], topo.edges[dofs_i, 1]
            self.tets.append(tets_i)
            self.dofs.append(dofs_i)
            self.w.append((om[ea] + om[eb]).astype(np.int64))
            self.vlayer.append(layer)
        wsum = np.zeros(topo.ne, dtype=np.int64)
        for d, w in zip(self.dofs, self.w):
            wsum[d] += w
        if np.any(wsum <= 0):
            raise RuntimeError("partition of unity has an uncovered edge")
        self.wsum = wsum
        self.D = [w / wsum[d] for d, w in zip(self.dofs, self.w)]
        self.dof_ptr = np.r_[0, np.cumsum([len(d) for d in self.dofs])].astype(np.int64)
        self.colour = self._colour()

    def _colour(self):
        """Greedy colouring (index order, smallest free colour) of the graph in
        which two subdomains are adjacent when their DOF lists intersect."""
        rows = np.concatenate(self.dofs)
        cols = np.repeat(np.arange(self.nsub), [len(d) for d in self.dofs])
        S = sp.csr_matrix((np.ones(rows.shape[0]), (rows, cols)), shape=(self.topo.ne, self.nsub))
        adj = (S.T @ S).tocsr()
        col = np.full(self.nsub, -1, dtype=np.int64)
        for i in range(self.nsub):
            nb = adj.indices[adj.indptr[i]:adj.indptr[i + 1]]
            used = set(col[nb][col[nb] >= 0].tolist())
            c = 0
            while c in used:
                c += 1
            col[i] = c
        self.adjacency = adj
        return col

    def neighbours(self, i):
        a = self.adjacency
        nb = a.indices[a.indptr[i]:a.indptr[i + 1]]
        return np.sort(nb[nb != i])

    # ----------------------------------------------------------------------
    def interface_faces(self, i):
        """Faces of the overlapping subdomain i: (tet, local face) pairs on
        the artificial interface and on the outer boundary."""
        topo = self.topo
        inT = np.zeros(topo.nt, dtype=bool)
        inT[self.tets[i]] = True
        fo = topo.face_of[self.tets[i]]                       # [n,4] face ids
        cnt = np.bincount(topo.face_of.ravel(), minlength=topo.nfaces_total)
        # faces seen twice within the subdomain are interior to it
        cnt_in = np.bincount(fo.ravel(), minlength=topo.nfaces_total)
        tl = np.repeat(self.tets[i], 4)
        lf = np.tile(np.arange(4), len(self.tets[i]))
        f = fo.ravel()
        outer = cnt[f] == 1
        iface = (cnt[f] == 2) & (cnt_in[f] == 1)
        return (tl[iface], lf[iface]), (tl[outer], lf[outer])

    def local_matrix(self, i, eps, eps_kind, freq_hz, eps_b):
        """ORAS matrix B_i (scipy CSR, rows/cols in dofs_i order)."""
        topo = self.topo
        k0 = fem.k0_of(freq_hz)
        kb = fem.wavenumber(k0, eps_b)
        tets = self.tets[i]
        dofs = self.dofs[i]
        loc = np.full(topo.ne, -1, dtype=np.int64)
        loc[dofs] = np.arange(len(dofs))
        sub = fem.Topology.__new__(fem.Topology)
        sub.xyz = topo.xyz
        sub.tet_sorted = topo.tet_sorted[tets]
        eps_arr = np.asarray(eps, dtype=np.complex128)
        e_t = eps_arr[tets] if eps_kind == 0 else eps_arr
        Ae = fem.element_operator(sub, e_t, eps_kind, k0)
        le = loc[topo.t2e[tets]]
        rows = [np.repeat(le, 6, axis=1).ravel()]
        cols = [np.tile(le, (1, 6)).ravel()]
        vals = [Ae.reshape(-1)]
        (it, il), (ot, ol) = self.interface_faces(i)
        lf = np.array(fem.LOCAL_FACES)
        lemap = {e: k for k, e in enumerate(fem.LOCAL_EDGES)}
        fe = np.array([[lemap[(f[p], f[q])] for (p, q) in fem.FACE_EDGES] for f in fem.LOCAL_FACES])
        epsT = fem.tet_eps(topo, eps_arr, eps_kind)
        for tt, ll, kk in ((it, il, fem.wavenumber(k0, epsT[it])), (ot, ol, np.full(len(ot), kb))):
            if len(tt) == 0:
                continue
            P = topo.xyz[topo.tet_sorted[tt[:, None], lf[ll]]]
            Bf = 1j * np.asarray(kk)[:, None, None] * fem.face_matrix(P)
            fl = loc[topo.t2e[tt[:, None], fe[ll]]]
            rows.append(np.repeat(fl, 3, axis=1).ravel())
            cols.append(np.tile(fl, (1, 3)).ravel())
            vals.append(Bf.reshape(-1))
        n = len(dofs)
        return sp.csr_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))),
                             shape=(n, n))


class ORAS:
    """M^{-1} v = sum_i R_i^T D_i B_i^{-1} R_i v with exact local solves.

    precision 'c128' factors B_i in complex128; 'c64' rounds B_i to complex64,
    factors it in complex64 and casts the restricted vector to complex64 and
    the local solution back (the mixed-precision preconditioner).
    """

    def __init__(self, dec: Decomposition, eps, eps_kind, freq_hz, eps_b,
                 precision: str = "c128", dense: bool | None = None):
        self.dec = dec
        self.precision = precision
        self.factors = []
        for i in range(dec.nsub):
            B = dec.local_matrix(i, eps, eps_kind, freq_hz, eps_b)
            use_dense = dense if dense is not None else B.shape[0] <= 3000
            if precision == "c64":
                Bd = B.toarray().astype(np.complex64)
                self.factors.append(("dense", sla.lu_factor(Bd, check_finite=False)))
            elif use_dense:
                self.factors.append(("dense", sla.lu_factor(B.toarray(), check_finite=False)))
            else:
                self.factors.append(("sparse", fem.sparse_lu(B)))

    def local_solve(self, i, x):
        kind, f = self.factors[i]
        if self.precision == "c64":
            return sla.lu_solve(f, x.astype(np.complex64), check_finite=False).astype(np.complex128)
        if kind == "dense":
            return sla.lu_solve(f, x, check_finite=False)
        return f.solve(np.asarray(x, dtype=np.complex128))

    def apply(self, v):
        v = np.asarray(v)
        z = np.zeros_like(v, dtype=np.complex128)
        for i in range(self.dec.nsub):
            d = self.dec.dofs[i]
            zi = self.local_solve(i, v[d])
            Di = self.dec.D[i]
            z[d] += (Di[:, None] * zi) if v.ndim == 2 else Di * zi
        return z
