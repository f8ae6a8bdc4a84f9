"""Port boundary conditions of the oracle (eq. (1), (3)) against closed
forms on a straight rectangular waveguide: the TE10 wave leaves port 0 and
arrives at port 1 as e^{-j beta L} with no reflection; the discrete result
converges to it at second order, is reciprocal, and conserves power when
the filling is lossless."""
import numpy as np
import pytest

import workload
from oracle import fem, ports

A_, B_, L_ = 0.03, 0.015, 0.06
F = 1e9


def _solve(n, eps):
    xyz, tet, pts = ports.waveguide(A_, B_, L_, n, eps)
    t = fem.Topology(xyz, tet)
    epsv = np.full(t.nt, eps)
    A, fp, pe = ports.assemble(t, epsv, 0, F, eps, pts, pec=True)
    B = ports.port_rhs(t, pts, fp, pe, F)
    U = fem.solve_direct(A, B)
    R = ports.port_functionals(t, pts, fp, pe)
    return t, pts, fp, pe, ports.scattering(R, U), R


def test_port_faces_and_metallic_edges():
    n = (6, 3, 8)
    xyz, tet, pts = ports.waveguide(A_, B_, L_, n, 44.0)
    t = fem.Topology(xyz, tet)
    fp = ports.classify(t, pts)
    assert (fp == 0).sum() == 2 * n[0] * n[1] and (fp == 1).sum() == 2 * n[0] * n[1]
    pe = ports.pec_edges(t, fp, True)
    # every edge on the four walls is metallic, and no interior port edge is
    wall = np.zeros(t.ne, bool)
    xa, xb = t.xyz[t.edges[:, 0]], t.xyz[t.edges[:, 1]]
    for ax, hi in ((0, A_), (1, B_)):
        for v in (0.0, hi):
            wall |= (np.abs(xa[:, ax] - v) < 1e-12) & (np.abs(xb[:, ax] - v) < 1e-12)
    assert np.array_equal(np.sort(pe), np.nonzero(wall)[0])


@pytest.mark.parametrize("eps", [44.0, 44.0 - 10.785j])
def test_straight_waveguide_converges_to_closed_form(eps):
    k0 = fem.k0_of(F)
    beta = ports.beta(k0, ports.Port((0, 0, 0), (0, 0, 1), (1, 0, 0), A_, B_, eps))
    exact = np.exp(-1j * beta * L_)
    errs = []
    for n in ((6, 3, 12), (12, 6, 24)):
        _, _, _, _, S, _ = _solve(n, eps)
        errs.append(abs(S[1, 0] - exact) + abs(S[0, 0]))
        assert abs(S[1, 0] - S[0, 1]) <= 1e-9 * abs(S[1, 0])
    print("errors", errs, "beta", beta)
    assert errs[1] <= 0.05
    assert errs[0] / errs[1] >= 2.5


def test_lossless_power_balance():
    _, _, _, _, S, _ = _solve((12, 6, 24), 44.0)
    p = abs(S[0, 0]) ** 2 + abs(S[1, 0]) ** 2
    assert abs(p - 1.0) <= 0.02


def test_receiver_normalisation():
    """The receiver functional of a port applied to the interpolated TE10
    field of that port gives 1 (normalisation of eq. (3))."""
    n = (12, 6, 24)
    xyz, tet, pts = ports.waveguide(A_, B_, L_, n, 44.0)
    t = fem.Topology(xyz, tet)
    fp = ports.classify(t, pts)
    pe = ports.pec_edges(t, fp, True)
    R = ports.port_functionals(t, pts, fp, pe)
    u0 = fem.edge_interpolant(t, lambda x: ports.mode(pts[0], x).astype(complex))
    assert abs(R[:, 0] @ u0 - 1.0) <= 2e-2


def test_box_chamber_apertures():
    """The generated port chamber: every aperture is covered by whole boundary
    faces (5 x 2 lattice cells = 20 triangles), apertures do not overlap, the
    field direction v = n x u is vertical, and reciprocity holds on a coarse
    lattice with the phantom inside."""
    xyz, tet, pts = workload.box_chamber(0.24, 0.2, 0.03, 1, (0.25, 0.75))
    t = fem.Topology(xyz, tet)
    fp = ports.classify(t, pts)
    assert len(pts) == 8 and np.array_equal(np.bincount(fp[fp >= 0], minlength=8), np.full(8, 20))
    for p in pts:
        v = np.cross(p.normal, p.u)
        assert np.allclose(v, (0, 0, 1))
    with pytest.raises(ValueError):
        workload.box_chamber(0.24, 0.2, 0.03, 2)       # two 5-cell apertures on an 8-cell wall
    lab = workload.shoulder_phantom(0).labels(workload.tet_centroids(xyz, tet))
    eps = workload.eps_of_labels(lab, F)
    eb = workload.eps_r(*workload.MATERIALS["matching"], F)
    A, fp, pe = ports.assemble(t, eps, 0, F, eb, pts, pec=True)
    U = fem.solve_direct(A, ports.port_rhs(t, pts, fp, pe, F))
    S = ports.scattering(ports.port_functionals(t, pts, fp, pe), U)
    assert np.abs(S - S.T).max() <= 1e-10 * np.abs(S).max()
