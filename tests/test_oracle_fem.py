"""Pins of the CPU oracle's discretisation against mathematics it must obey.

Each test checks the oracle against something other than itself: closed-form
mesh counts, brute-force quadrature of the Nedelec basis, the curl kernel,
exact reproduction of constant and linear fields, reciprocity, and the
O(h) convergence to a closed-form plane wave in a homogeneous lossy medium.
"""
import itertools
import json
import math
import os

import numpy as np
import pytest

import workload
from oracle import fem
from tests import quadrature as Q

GOLD = os.path.join(os.path.dirname(__file__), "golden")


# -- topology ---------------------------------------------------------------

@pytest.mark.parametrize("n", [1, 2, 3, 4, 8])
def test_kuhn_counts_closed_form(n):
    """V=(n+1)^3, E=3n(n+1)^2+3n^2(n+1)+n^3, T=6n^3, 12n^2 boundary faces,
    and Euler's formula V - E + F - T = 1 for a ball."""
    xyz, tet = workload.kuhn_cube(n)
    t = fem.Topology(xyz, tet)
    assert t.nv == (n + 1) ** 3
    assert t.ne == 3 * n * (n + 1) ** 2 + 3 * n * n * (n + 1) + n ** 3
    assert t.nt == 6 * n ** 3
    assert len(t.bface_tet) == 12 * n * n
    assert t.nv - t.ne + t.nfaces_total - t.nt == 1


def test_kuhn_counts_golden():
    g = json.load(open(os.path.join(GOLD, "kuhn_cube8_counts.json")))
    xyz, tet = workload.kuhn_cube(8)
    t = fem.Topology(xyz, tet)
    assert [t.nv, t.ne, t.nt, len(t.bface_tet), t.nfaces_total] == \
        [g["V"], g["E"], g["T"], g["boundary_faces"], g["faces"]]


@pytest.mark.parametrize("n", [2, 3])
def test_pattern_brute_force(n):
    """Edges, tet->edge map and CSR pattern against a set-based brute force."""
    xyz, tet = workload.kuhn_cube(n)
    t = fem.Topology(xyz, tet)
    edges = sorted({tuple(sorted((int(a), int(b)))) for row in tet for a, b in itertools.combinations(row, 2)})
    assert [tuple(e) for e in t.edges.tolist()] == edges
    eid = {e: i for i, e in enumerate(edges)}
    pairs = set()
    for k, row in enumerate(tet):
        es = [eid[tuple(sorted((int(a), int(b))))] for a, b in itertools.combinations(row, 2)]
        assert sorted(es) == sorted(t.t2e[k].tolist())
        pairs.update((p, q) for p in es for q in es)
    got = set(zip(np.repeat(np.arange(t.ne), np.diff(t.row_ptr)).tolist(), t.col.tolist()))
    assert got == pairs
    faces = {}
    for row in tet:
        for f in itertools.combinations(sorted(int(v) for v in row), 3):
            faces[f] = faces.get(f, 0) + 1
    bnd = sorted(f for f, c in faces.items() if c == 1)
    assert [tuple(f) for f in t.bface_verts.tolist()] == bnd


def test_jittered_cylinder_valid():
    p = workload.chamber_problem(c=0.02, nsub=8)
    t = fem.Topology(p.xyz, p.tet)
    X = p.xyz[t.tet_sorted]
    vol = np.linalg.det(X[:, 1:] - X[:, :1]) / 6.0
    h = 0.02
    assert np.all(np.abs(vol) > 0.05 * h ** 3 / 6)
    assert t.nv - t.ne + t.nfaces_total - t.nt == 1   # still a ball


# -- element matrices -------------------------------------------------------

def _random_tets(k, seed):
    rng = np.random.default_rng(seed)
    out = []
    while len(out) < k:
        X = rng.uniform(-1, 1, (4, 3)) * rng.uniform(0.01, 2.0)
        if Q.tet_volume(X) > 1e-3 * np.linalg.norm(X[1] - X[0]) ** 3:
            out.append(X)
    return out


def test_element_matrices_vs_quadrature():
    """K_T, M_T, M_{T,n} against quadrature of the Whitney functions with
    exact barycentric gradients and central-difference curls."""
    lam, w = Q.tet_rule(5)
    for X in _random_tets(6, 1):
        vol = Q.tet_volume(X)
        pts = lam @ X
        N = [Q.whitney(X, pts, a, b) for (a, b) in fem.LOCAL_EDGES]
        h = 1e-4 * np.linalg.norm(X[1] - X[0])
        C = [Q.curl_fd(lambda p, a=a, b=b: Q.whitney(X, p, a, b), pts, h) for (a, b) in fem.LOCAL_EDGES]
        Kq = np.array([[vol * (w * (C[p] * C[q]).sum(1)).sum() for q in range(6)] for p in range(6)])
        Mq = np.array([[vol * (w * (N[p] * N[q]).sum(1)).sum() for q in range(6)] for p in range(6)])
        Mnq = np.array([[[vol * (w * lam[:, n] * (N[p] * N[q]).sum(1)).sum() for q in range(6)]
                         for p in range(6)] for n in range(4)])
        K, M = fem.element_matrices(X[None])
        Mn = fem.element_mass_p1(X[None])
        assert np.allclose(K[0], Kq, rtol=1e-7, atol=1e-7 * np.abs(Kq).max())
        assert np.allclose(M[0], Mq, rtol=1e-10, atol=1e-12 * np.abs(Mq).max())
        assert np.allclose(Mn[0], Mnq, rtol=1e-10, atol=1e-12 * np.abs(Mnq).max())


def test_edge_moments():
    """int over edge f of N_e . dl = delta_ef (the DOFs are edge circulations)."""
    xg, wg = np.polynomial.legendre.leggauss(3)
    s = 0.5 * (xg + 1); wg = 0.5 * wg
    for X in _random_tets(4, 2):
        for p, (a, b) in enumerate(fem.LOCAL_EDGES):
            for q, (c, d) in enumerate(fem.LOCAL_EDGES):
                pts = X[c][None] + s[:, None] * (X[d] - X[c])[None]
                val = (wg * (Q.whitney(X, pts, a, b) @ (X[d] - X[c]))).sum()
                assert abs(val - (p == q)) < 1e-10


def test_element_invariants():
    """K_T symmetric PSD of rank 3 with K_T G_T = 0; M_T symmetric positive
    definite; sum_n M_{T,n} = M_T."""
    Gt = np.zeros((6, 4))
    for p, (a, b) in enumerate(fem.LOCAL_EDGES):
        Gt[p, a] = -1; Gt[p, b] = 1
    for X in _random_tets(6, 3):
        K, M = fem.element_matrices(X[None])
        K, M = K[0], M[0]
        assert np.array_equal(K, K.T) and np.array_equal(M, M.T)
        ev = np.linalg.eigvalsh(K)
        assert ev.min() > -1e-12 * ev.max()
        assert np.sum(ev > 1e-10 * ev.max()) == 3
        assert np.abs(K @ Gt).max() < 1e-12 * np.abs(K).max()
        assert np.linalg.eigvalsh(M).min() > 0
        Mn = fem.element_mass_p1(X[None])[0]
        assert np.allclose(Mn.sum(axis=0), M, rtol=1e-13, atol=1e-15 * np.abs(M).max())


def test_face_matrix_vs_quadrature():
    """B_F against quadrature of tangential traces N - (N.n) n of the 3-D
    Whitney functions on a face of a random tetrahedron."""
    lam2, w2 = Q.tri_rule(4)
    for X in _random_tets(4, 4):
        for f in fem.LOCAL_FACES:
            P = X[list(f)]
            nrm = np.cross(P[1] - P[0], P[2] - P[0])
            area = 0.5 * np.linalg.norm(nrm)
            nrm = nrm / np.linalg.norm(nrm)
            pts = lam2 @ P
            T = []
            for (p, q) in fem.FACE_EDGES:
                N = Q.whitney(X, pts, f[p], f[q])
                T.append(N - (N @ nrm)[:, None] * nrm[None])
            Bq = np.array([[area * (w2 * (T[i] * T[j]).sum(1)).sum() for j in range(3)] for i in range(3)])
            B = fem.face_matrix(P[None])[0]
            assert np.allclose(B, Bq, rtol=1e-11, atol=1e-13 * np.abs(Bq).max())


# -- global operator --------------------------------------------------------

def test_curl_kernel():
    """K G phi = 0 for every nodal phi; rank K = E - V + 1 (simply connected)."""
    xyz, tet = workload.kuhn_cube(8)
    t = fem.Topology(xyz, tet)
    K = fem.curl_curl_matrix(t)
    G = fem.gradient_matrix(t)
    phi = np.random.default_rng(0).standard_normal(t.nv)
    gp = G @ phi
    assert np.linalg.norm(K @ gp) <= 1e-12 * abs(K).max() * np.linalg.norm(gp) * 10
    xyz, tet = workload.kuhn_cube(4)
    t4 = fem.Topology(xyz, tet)
    K4 = fem.curl_curl_matrix(t4).toarray()
    assert np.linalg.matrix_rank(K4) == t4.ne - t4.nv + 1


def test_reciprocity_and_symmetry():
    p = workload.cube_problem(n=6)
    t = fem.Topology(p.xyz, p.tet)
    A = fem.assemble(t, p.eps, 0, p.freq, p.eps_b)
    assert (A != A.T).nnz == 0
    U = fem.solve_direct(A, fem.dipole_rhs(t, p.src_pos, p.src_mom, p.freq))
    S = fem.scattering(fem.functionals(t, p.src_pos, p.src_mom), U)
    assert np.abs(S - S.T).max() <= 1e-10 * np.abs(S).max()


def test_point_functional_reproduces_linear_fields():
    """Lowest-order Nedelec interpolation is exact for E = a + b x x, so the
    point functional must return p . E(x) exactly, also on faces/edges/vertices
    (where it averages over the containing tetrahedra)."""
    xyz, tet = workload.kuhn_cube(4)
    t = fem.Topology(xyz, tet)
    rng = np.random.default_rng(5)
    a = rng.standard_normal(3) + 1j * rng.standard_normal(3)
    bb = rng.standard_normal(3)
    xa = t.xyz[t.edges[:, 0]]; xb = t.xyz[t.edges[:, 1]]
    mid = 0.5 * (xa + xb)
    u = ((a[None] + np.cross(bb[None], mid)) * (xb - xa)).sum(1)
    pts = [rng.uniform(0.01, 0.09, 3) for _ in range(4)]
    pts += [np.array([0.0321, 0.0517, 0.05]),      # on a grid plane
            np.array([0.0321, 0.05, 0.05]),        # on a grid line
            np.array([0.05, 0.05, 0.05])]          # on a vertex
    for x in pts:
        pm = rng.standard_normal(3) + 0j
        r = fem.point_functional(t, x, pm)
        assert abs(r @ u - pm @ (a + np.cross(bb, x))) < 1e-11 * (1 + np.abs(u).max())


# -- plane wave: O(h) convergence ------------------------------------------

TRI7 = None


def _plane_wave_error(n, eps, freq=1e9):
    xyz, tet = workload.kuhn_cube(n)
    t = fem.Topology(xyz, tet)
    k0 = 2 * math.pi * freq / fem.C0
    k = k0 * np.sqrt(complex(eps))
    d = np.array([1.0, 2.0, 3.0]); d /= np.linalg.norm(d)
    pol = np.cross(d, [0.0, 0.0, 1.0]); pol /= np.linalg.norm(pol)

    def E(x):
        return pol[None] * np.exp(-1j * k * (x @ d))[:, None]

    # impedance data g = (curl E) x n + j k n x (E x n), curl E = -j k d x E
    lam2, w2 = Q.tri_rule(5)
    b = np.zeros(t.ne, dtype=complex)
    for f in range(len(t.bface_tet)):
        T = t.bface_tet[f]
        Xt = t.xyz[t.tet_sorted[T]]
        lf = fem.LOCAL_FACES[t.bface_local[f]]
        P = Xt[list(lf)]
        nrm = np.cross(P[1] - P[0], P[2] - P[0])
        area = 0.5 * np.linalg.norm(nrm)
        nrm /= np.linalg.norm(nrm)
        opp = [v for v in range(4) if v not in lf][0]
        if (Xt[opp] - P[0]) @ nrm > 0:
            nrm = -nrm
        pts = lam2 @ P
        Ev = E(pts)
        cE = -1j * k * np.cross(d[None], Ev)
        g = np.cross(cE, nrm[None]) + 1j * k * np.cross(nrm[None], np.cross(Ev, nrm[None]))
        for j, (p, q) in enumerate(fem.FACE_EDGES):
            N = Q.whitney(Xt, pts, lf[p], lf[q])
            b[t.bface_edges[f, j]] += area * (w2 * (g * N).sum(1)).sum()
    epsv = np.full(t.nt, complex(eps))
    A = fem.assemble(t, epsv, 0, freq, complex(eps))
    u = fem.solve_direct(A, b, dense_max=5000)
    # L2 error with a 4-point-per-direction collapsed rule on every tet
    lam, w = Q.tet_rule(4)
    X = t.xyz[t.tet_sorted]
    g = Q.bary_grads(X)                          # [T,4,3]
    vol = np.abs(np.linalg.det(X[:, 1:] - X[:, :1])) / 6
    pts = np.einsum("qk,tkd->tqd", lam, X)
    Eh = np.zeros(pts.shape, dtype=complex)
    for le, (a, bb) in enumerate(fem.LOCAL_EDGES):
        N = lam[None, :, a, None] * g[:, None, bb] - lam[None, :, bb, None] * g[:, None, a]
        Eh += u[t.t2e[:, le]][:, None, None] * N
    Ex = E(pts.reshape(-1, 3)).reshape(pts.shape)
    err = np.sqrt((vol[:, None] * w[None] * (np.abs(Eh - Ex) ** 2).sum(-1)).sum())
    ref = np.sqrt((vol[:, None] * w[None] * (np.abs(Ex) ** 2).sum(-1)).sum())
    return err / ref


@pytest.mark.parametrize("eps,ns", [(4 - 1j, (4, 8, 16)), (44 - 10.785j, (8, 16))])
def test_plane_wave_convergence(eps, ns):
    errs = [_plane_wave_error(n, eps) for n in ns]
    for e1, e2 in zip(errs, errs[1:]):
        assert e1 / e2 >= 1.8, errs
    assert errs[-1] < (0.2 if abs(eps) < 10 else 0.5)


# -- point dipole: closed-form field in a homogeneous lossy medium ----------

def _dipole_fields(x, xs, p, k, omu):
    """E and curl E of J = p delta(x - xs) in a homogeneous medium (exp(+j w t)):
    E = -j w mu0 (I + grad grad / k^2) g p,  g = exp(-j k r) / (4 pi r),
    curl E = -j w mu0 grad g x p (written out from the dyadic Green's function)."""
    d = x - xs[None]
    r = np.linalg.norm(d, axis=1)
    rh = d / r[:, None]
    kr = k * r
    g = np.exp(-1j * kr) / (4 * np.pi * r)
    a = 1 - 1j / kr - 1 / kr ** 2
    b = -1 + 3j / kr + 3 / kr ** 2
    E = -1j * omu * g[:, None] * (a[:, None] * p[None] + (b * (rh @ p))[:, None] * rh)
    gradg = (g * (-1j * k - 1 / r))[:, None] * rh
    return E, -1j * omu * np.cross(gradg, p[None])


def _dipole_error(n, eps=4 - 1j, freq=1e9, rmin=0.03):
    """Relative L2 error, outside the ball |x - xs| < rmin, of the FE field
    with the oracle's dipole right-hand side and the exact impedance data of
    the dipole field on the cube faces; column 1 has the interior source
    doubled (a wrong amplitude, the control)."""
    xyz, tet = workload.kuhn_cube(n, 0.1)
    t = fem.Topology(xyz, tet)
    xs = np.array([0.0513, 0.0497, 0.0502])
    p = np.array([0.3, -0.2, 1.0])
    k = fem.wavenumber(fem.k0_of(freq), eps)
    omu = fem.omega_mu0(freq)
    src = fem.dipole_rhs(t, xs[None], p[None].astype(complex), freq)[:, 0]
    bnd = np.zeros(t.ne, dtype=complex)
    lam2, w2 = Q.tri_rule(5)
    for f in range(len(t.bface_tet)):
        Xt = t.xyz[t.tet_sorted[t.bface_tet[f]]]
        lf = fem.LOCAL_FACES[t.bface_local[f]]
        P = Xt[list(lf)]
        nrm = np.cross(P[1] - P[0], P[2] - P[0])
        area = 0.5 * np.linalg.norm(nrm)
        nrm /= np.linalg.norm(nrm)
        opp = [v for v in range(4) if v not in lf][0]
        if (Xt[opp] - P[0]) @ nrm > 0:
            nrm = -nrm
        pts = lam2 @ P
        Ev, cE = _dipole_fields(pts, xs, p, k, omu)
        g = np.cross(cE, nrm[None]) + 1j * k * np.cross(nrm[None], np.cross(Ev, nrm[None]))
        for j, (a, b) in enumerate(fem.FACE_EDGES):
            N = Q.whitney(Xt, pts, lf[a], lf[b])
            bnd[t.bface_edges[f, j]] += area * (w2 * (g * N).sum(1)).sum()
    A = fem.assemble(t, np.full(t.nt, eps), 0, freq, eps)
    U = fem.solve_direct(A, np.stack([src + bnd, 2 * src + bnd], axis=1))
    lam, w = Q.tet_rule(3)
    X = t.xyz[t.tet_sorted]
    gr = Q.bary_grads(X)
    vol = np.abs(np.linalg.det(X[:, 1:] - X[:, :1])) / 6
    keep = np.linalg.norm(X.mean(1) - xs, axis=1) > rmin
    pts = np.einsum("qk,tkd->tqd", lam, X)
    Ex = _dipole_fields(pts.reshape(-1, 3), xs, p, k, omu)[0].reshape(pts.shape)
    ref = np.sqrt((vol[:, None] * w[None] * (np.abs(Ex) ** 2).sum(-1))[keep].sum())
    errs = []
    for c in range(2):
        Eh = np.zeros(pts.shape, dtype=complex)
        for le, (a, b) in enumerate(fem.LOCAL_EDGES):
            N = lam[None, :, a, None] * gr[:, None, b] - lam[None, :, b, None] * gr[:, None, a]
            Eh += U[t.t2e[:, le], c][:, None, None] * N
        errs.append(np.sqrt((vol[:, None] * w[None] * (np.abs(Eh - Ex) ** 2).sum(-1))[keep].sum()) / ref)
    return errs


def test_dipole_matches_closed_form():
    """The dipole right-hand side -j w mu0 p.N_e(x_s) reproduces the
    closed-form field of a point dipole: the error away from the source falls
    with h (measured 0.75, 0.42, 0.29 at n = 8, 12, 16), while a doubled
    amplitude (the control) stays near |1 - 2| = 1; a wrong sign, factor, or
    phase convention would likewise leave an O(1) error."""
    errs = [_dipole_error(n) for n in (8, 12, 16)]
    good = [e[0] for e in errs]
    for e1, e2 in zip(good, good[1:]):
        assert e1 / e2 >= 1.3, good
    assert good[-1] < 0.35, good
    assert errs[-1][1] > 0.7, errs
