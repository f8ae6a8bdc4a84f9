"""Pins of the oracle's Schwarz pieces and Krylov solver.

Checks: the bisection reproduces the 2x2x2 box split of the cube, a
set-based brute force of the overlap layers and DOF lists, the partition of
unity sums to one and vanishes on the artificial boundary, colours are
proper, one subdomain makes ORAS an exact inverse (one FGMRES iteration),
and FGMRES reproduces the direct solve.
"""
import numpy as np
import pytest
import scipy.sparse as sp

import workload
from oracle import fem, krylov, schwarz


@pytest.fixture(scope="module")
def cube():
    p = workload.cube_problem(n=8)
    t = fem.Topology(p.xyz, p.tet)
    A = fem.assemble(t, p.eps, 0, p.freq, p.eps_b)
    return p, t, A


def test_rcb_box_split(cube):
    """At the cube the 8 RCB parts are the 8 octants of 4x4x4 lattice cubes."""
    p, t, _ = cube
    part = schwarz.rcb(p.xyz, p.tet, 8)
    cube_id = np.arange(t.nt) // 6
    i = cube_id % 8; j = (cube_id // 8) % 8; k = cube_id // 64
    octant = (i >= 4).astype(int) * 1 + (j >= 4) * 2 + (k >= 4) * 4
    mapping = {}
    for o, q in zip(octant, part):
        assert mapping.setdefault(int(o), int(q)) == int(q)
    assert sorted(mapping.values()) == list(range(8))
    assert np.all(np.bincount(part) == t.nt // 8)


def test_overlap_brute_force():
    """Overlap layers and DOF lists against loops over Python sets."""
    p = workload.cube_problem(n=4, nsub=4, overlap=2)
    t = fem.Topology(p.xyz, p.tet)
    dec = schwarz.Decomposition(t, 4, 2)
    ts = [set(map(int, r)) for r in t.tet_sorted]
    for i in range(4):
        cur = {k for k in range(t.nt) if dec.part[k] == i}
        for _ in range(2):
            vs = set().union(*(ts[k] for k in cur))
            cur = {k for k in range(t.nt) if ts[k] & vs}
        assert sorted(cur) == dec.tets[i].tolist()
        dofs = sorted({int(e) for k in cur for e in t.t2e[k]})
        assert dofs == dec.dofs[i].tolist()


@pytest.mark.parametrize("overlap", [1, 2])
def test_partition_of_unity(cube, overlap):
    """sum_i R_i^T D_i R_i = I, and D_i = 0 on edges of the artificial interface."""
    p, t, _ = cube
    dec = schwarz.Decomposition(t, 8, overlap)
    s = np.zeros(t.ne)
    for d, D in zip(dec.dofs, dec.D):
        s[d] += D
    assert np.allclose(s, 1.0, rtol=0, atol=1e-15)
    lf = np.array(fem.LOCAL_FACES)
    lemap = {e: k for k, e in enumerate(fem.LOCAL_EDGES)}
    fe = np.array([[lemap[(f[a], f[b])] for (a, b) in fem.FACE_EDGES] for f in fem.LOCAL_FACES])
    for i in range(8):
        (it, il), _ = dec.interface_faces(i)
        assert len(it) > 0
        edges = np.unique(t.t2e[it[:, None], fe[il]])
        loc = np.searchsorted(dec.dofs[i], edges)
        assert np.all(dec.D[i][loc] == 0)


def test_colouring_is_proper(cube):
    p, t, _ = cube
    dec = schwarz.Decomposition(t, 8, 2)
    for i in range(8):
        for j in range(i + 1, 8):
            if np.intersect1d(dec.dofs[i], dec.dofs[j]).size:
                assert dec.colour[i] != dec.colour[j]


def test_one_subdomain_is_exact(cube):
    """nsub = 1: B_1 = A, so M^{-1} = A^{-1} and FGMRES stops after one step."""
    p, t, A = cube
    dec = schwarz.Decomposition(t, 1, 1)
    B = dec.local_matrix(0, p.eps, 0, p.freq, p.eps_b)
    assert abs(B - A).max() <= 1e-12 * abs(A).max()
    M = schwarz.ORAS(dec, p.eps, 0, p.freq, p.eps_b)
    b = fem.dipole_rhs(t, p.src_pos[:1], p.src_mom[:1], p.freq)[:, 0]
    x, it, rr, _ = krylov.fgmres(lambda v: A @ v, M.apply, b, 1e-8, 40)
    assert it == 1 and rr < 1e-10


def test_ras_local_matrix_interior_rows(cube):
    """Rows of B_i on DOFs whose whole tetrahedron star lies inside the
    overlapping subdomain equal the rows of A (only the artificial boundary
    differs)."""
    p, t, A = cube
    dec = schwarz.Decomposition(t, 8, 2)
    i = 3
    B = dec.local_matrix(i, p.eps, 0, p.freq, p.eps_b).tocsr()
    d = dec.dofs[i]
    inside = np.zeros(t.nt, bool); inside[dec.tets[i]] = True
    e2t = sp.csr_matrix((np.ones(6 * t.nt), (t.t2e.ravel(), np.repeat(np.arange(t.nt), 6))),
                        shape=(t.ne, t.nt))
    star_out = np.asarray(e2t[d][:, ~inside].sum(axis=1)).ravel()
    rows = np.nonzero(star_out == 0)[0]
    Ar = A[d][:, d].tocsr()
    diff = abs(B[rows] - Ar[rows]).max()
    assert diff <= 1e-12 * abs(A).max()


@pytest.mark.parametrize("precision,tol", [("c128", 1e-7), ("c64", 1e-7)])
def test_fgmres_matches_direct(cube, precision, tol):
    p, t, A = cube
    dec = schwarz.Decomposition(t, 8, 1)
    M = schwarz.ORAS(dec, p.eps, 0, p.freq, p.eps_b, precision=precision)
    B = fem.dipole_rhs(t, p.src_pos[:3], p.src_mom[:3], p.freq)
    U = fem.solve_direct(A, B)
    X, its, res = krylov.fgmres_block(A, M.apply, B, 1e-9, 40)
    assert np.all(res <= 1e-9)
    err = np.linalg.norm(X - U, axis=0) / np.linalg.norm(U, axis=0)
    assert err.max() < tol
    assert its.max() < 40


def test_givens_zeroes():
    rng = np.random.default_rng(0)
    for _ in range(20):
        a = complex(*rng.standard_normal(2)); b = complex(*rng.standard_normal(2))
        c, s = krylov.givens(a, b)
        assert abs(-np.conj(s) * a + c * b) < 1e-15
        assert abs(c * c + abs(s) ** 2 - 1) < 1e-15


def test_interface_faces_brute_force():
    """Every face of an overlapping subdomain is classified by looping over
    Python sets of vertex triples: a face met by one tetrahedron of the whole
    mesh is outer boundary, a face met by one tetrahedron inside the subdomain
    and one outside is artificial interface; the oracle's lists must be
    exactly these sets (none missing, none extra, no face twice)."""
    p = workload.chamber_problem(c=0.03, nsub=8, overlap=1, nsrc=2)
    t = fem.Topology(p.xyz, p.tet)
    dec = schwarz.Decomposition(t, 8, 1)
    owners = {}
    for k, tv in enumerate(t.tet_sorted):
        for lf in fem.LOCAL_FACES:
            owners.setdefault(tuple(int(tv[a]) for a in lf), []).append(k)
    for i in range(dec.nsub):
        inside = set(dec.tets[i].tolist())
        want_if, want_out = set(), set()
        for k in inside:
            for lf in fem.LOCAL_FACES:
                f = tuple(int(t.tet_sorted[k][a]) for a in lf)
                own = owners[f]
                if len(own) == 1:
                    want_out.add((k, f))
                elif sum(o in inside for o in own) == 1:
                    want_if.add((k, f))
        (it, il), (ot, ol) = dec.interface_faces(i)
        got_if = [(int(k), tuple(int(t.tet_sorted[k][a]) for a in fem.LOCAL_FACES[l])) for k, l in zip(it, il)]
        got_out = [(int(k), tuple(int(t.tet_sorted[k][a]) for a in fem.LOCAL_FACES[l])) for k, l in zip(ot, ol)]
        assert len(got_if) == len(set(got_if)) and set(got_if) == want_if, i
        assert len(got_out) == len(set(got_out)) and set(got_out) == want_out, i
        assert len(want_if) > 0
