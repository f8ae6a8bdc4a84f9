"""Waveguide-port chamber (metallic box, ceramic-filled apertures on two rings,
shoulder phantom inside) on the GPU path against the oracle.

Small lattice (3.7k edges, 8 ports): fields and scattering matrix against the
oracle's direct solve of the port system. Full size (1.16M edges, 32 ports,
the measured launch configuration: 512 subdomains, one overlap layer,
complex64 factors): operator values to rounding over the whole mesh, and the
solution certified with the oracle's own operator, right-hand sides and
receiver functionals (true residual of every port, S = R^T E - I).
"""
import numpy as np
import pytest
import scipy.sparse as sp

from oracle import fem, ports

mx = pytest.importorskip("paper_2311_05322_amd")
from paper_2311_05322_amd.port_chamber import box_problem  # noqa: E402

pytestmark = pytest.mark.gpu
F = 1e9


def _oracle(xyz, tet, eps, eb, pts):
    t = fem.Topology(xyz, tet)
    A, fp, pe = ports.assemble(t, eps, 0, F, eb, pts, pec=True)
    B = ports.port_rhs(t, pts, fp, pe, F)
    R = ports.port_functionals(t, pts, fp, pe)
    return t, A, B, R, pe


def _ctx(xyz, tet, eps, eb, pts):
    ctx = mx.Context(0)
    ctx.assemble(xyz, tet, eps, mx.MX_EPS_P0, F, eb)
    ctx.set_ports(pts, pec=True)
    return ctx


def _operator_err(ctx, t, A):
    v = ctx.matrix_values()
    D = (sp.csr_matrix((v, t.col, t.row_ptr), shape=(t.ne, t.ne)) - A).tocoo()
    return (np.abs(D.data).max() if D.nnz else 0.0) / np.abs(A.data).max()


@pytest.mark.parametrize("prec,tol", [(mx.MX_PREC_C128, 1e-6), (mx.MX_PREC_C64, 1e-5)], ids=["c128", "c64"])
def test_small_box_chamber_matches_direct(prec, tol):
    print("[case] box chamber h=30 mm, 8 ports", flush=True)
    xyz, tet, eps, eb, pts = box_problem(0.03, 1, rings=(0.25, 0.75))
    t, A, B, R, pe = _oracle(xyz, tet, eps, eb, pts)
    U = fem.solve_direct(A, B)
    S_ref = ports.scattering(R, U)
    ctx = _ctx(xyz, tet, eps, eb, pts)
    try:
        assert _operator_err(ctx, t, A) <= 1e-13
        ctx.setup_schwarz(8, 1, precision=prec)
        E, S, info = ctx.solve_ports(rtol=1e-10 if prec == mx.MX_PREC_C128 else 1e-8)
        print("iters", info["iters"], flush=True)
        assert info["converged"]
        err = np.linalg.norm(E - U, axis=0) / np.linalg.norm(U, axis=0)
        assert err.max() <= tol, err
        assert np.abs(S - S_ref).max() <= 10 * tol * np.abs(S_ref).max()
        assert np.abs(S - S.T).max() <= 10 * tol * np.abs(S).max()
    finally:
        ctx.close()


@pytest.mark.slow
@pytest.mark.timeout(600)
def test_fullsize_port_chamber_certified():
    print("[case] box chamber h=4.2 mm (1.16M edges), 32 ports, nsub=512 overlap=1 c64", flush=True)
    xyz, tet, eps, eb, pts = box_problem(0.0042, 4)
    ctx = _ctx(xyz, tet, eps, eb, pts)
    try:
        ctx.setup_schwarz(512, 1, precision=mx.MX_PREC_C64)
        E, S, info = ctx.solve_ports(rtol=1e-8)
        print("iters", info["iters_max"], "relres", info["relres"].max(), flush=True)
        assert info["converged"] and len(pts) == 32
        print("[oracle] assembling the port system", flush=True)
        t, A, B, R, pe = _oracle(xyz, tet, eps, eb, pts)
        assert t.ne == E.shape[0] == 1157264
        assert _operator_err(ctx, t, A) <= 1e-13
        res = np.linalg.norm(B - A @ E, axis=0) / np.linalg.norm(B, axis=0)
        print("true residuals", res.max(), flush=True)
        assert res.max() <= 1.5e-8
        assert np.abs(E[pe]).max() == 0.0
        S_o = ports.scattering(R, E)
        assert np.abs(S - S_o).max() <= 1e-10 * np.abs(S_o).max()
        assert np.abs(S - S.T).max() <= 1e-5 * np.abs(S).max()
    finally:
        ctx.close()
