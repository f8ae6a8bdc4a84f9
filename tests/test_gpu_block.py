"""Block FGMRES on the GPU path (mx_set_krylov: one-pass block Gram-Schmidt
with a second pass only where a column lost accuracy, and the always-two-pass
variant) against the oracle: the fields
of the direct solve (1e-6 with complex128 factors, 1e-5 with complex64), the
oracle's block FGMRES step count with the same ORAS preconditioner, the
single-column case equal to the pseudo-block solver, groups of at most 32
columns in lockstep for wider blocks, and the fallback to the pseudo-block
solver for a zero or a repeated right-hand side."""
import numpy as np
import pytest

import workload
from oracle import block_krylov, fem, ports, schwarz

mx = pytest.importorskip("paper_2311_05322_amd")
pytestmark = pytest.mark.gpu


class Case:
    def __init__(self, name, two_pass=False):
        print(f"[case] {name} two_pass={two_pass}", flush=True)
        self.two_pass = two_pass
        if name == "cube8":
            self.p = workload.cube_problem(n=8)
        else:
            self.p = workload.chamber_problem(c=0.02, nsub=16, overlap=2, nsrc=8)
        p = self.p
        self.t = fem.Topology(p.xyz, p.tet)
        self.A = fem.assemble(self.t, p.eps, p.eps_kind, p.freq, p.eps_b)
        self.B = fem.dipole_rhs(self.t, p.src_pos, p.src_mom, p.freq)
        self.U = fem.solve_direct(self.A, self.B)
        self.ctx = mx.Context(0)
        self.ctx.assemble(p.xyz, p.tet, p.eps, p.eps_kind, p.freq, p.eps_b)
        self.ctx.set_krylov(True, two_pass)


@pytest.fixture(scope="module", params=[("cube8", False), ("cube8", True), ("chamber20", False), ("chamber20", True)],
                ids=["cube8-cgs1", "cube8-cgs2", "chamber20-cgs1", "chamber20-cgs2"])
def case(request):
    c = Case(*request.param)
    yield c
    c.ctx.close()


@pytest.mark.parametrize("prec,tol", [(mx.MX_PREC_C128, 1e-6), (mx.MX_PREC_C64, 1e-5)], ids=["c128", "c64"])
def test_block_fields_match_direct_solve(case, prec, tol):
    p = case.p
    case.ctx.setup_schwarz(p.nsub, p.overlap, precision=prec)
    E, S, info = case.ctx.solve(p.src_pos, p.src_mom, rtol=1e-10)
    print("block steps", info["iters_max"], "cycles", info["cycles"], "fallback", info["fallback"], flush=True)
    assert info["converged"] and info["fallback"] == 0
    assert np.all(info["relres"] <= 1e-10)
    err = np.linalg.norm(E - case.U, axis=0) / np.linalg.norm(case.U, axis=0)
    assert err.max() <= tol, err
    res = np.linalg.norm(case.B - case.A @ E, axis=0) / np.linalg.norm(case.B, axis=0)
    assert res.max() <= 1e-9


def test_block_steps_match_oracle(case):
    p = case.p
    case.ctx.setup_schwarz(p.nsub, p.overlap, precision=mx.MX_PREC_C128, restart=30)
    _, _, info = case.ctx.solve(p.src_pos, p.src_mom, rtol=1e-8, want_E=False)
    dec = schwarz.Decomposition(case.t, p.nsub, p.overlap)
    M = schwarz.ORAS(dec, p.eps, p.eps_kind, p.freq, p.eps_b)
    _, steps, rr, _ = block_krylov.block_fgmres(lambda V: case.A @ V, M.apply, case.B, 1e-8, 30)
    print("gpu block steps", info["iters_max"], "oracle block steps", steps, flush=True)
    assert abs(info["iters_max"] - steps) <= 1
    # the block space holds every column's own Krylov space
    case.ctx.set_krylov(False)
    try:
        _, _, info_pb = case.ctx.solve(p.src_pos, p.src_mom, rtol=1e-8, want_E=False)
    finally:
        case.ctx.set_krylov(True, case.two_pass)
    assert info["iters_max"] <= info_pb["iters_max"]


def test_one_column_equals_pseudo_block(case):
    p = case.p
    case.ctx.setup_schwarz(p.nsub, p.overlap, precision=mx.MX_PREC_C128)
    E1, _, info1 = case.ctx.solve(p.src_pos[:1], p.src_mom[:1], rtol=1e-10)
    case.ctx.set_krylov(False)
    try:
        E0, _, info0 = case.ctx.solve(p.src_pos[:1], p.src_mom[:1], rtol=1e-10)
    finally:
        case.ctx.set_krylov(True, case.two_pass)
    assert abs(info1["iters_max"] - info0["iters_max"]) <= 1
    assert np.linalg.norm(E1 - E0) <= 1e-8 * np.linalg.norm(E0)


def test_ragged_and_fallbacks():
    c = Case("cube8")
    p = c.p
    try:
        c.ctx.setup_schwarz(p.nsub, p.overlap, precision=mx.MX_PREC_C64)
        # 5 columns (a width that fills no 16-wide MFMA tile)
        E, _, info = c.ctx.solve(p.src_pos[:5], p.src_mom[:5], rtol=1e-9)
        assert info["converged"] and info["fallback"] == 0
        err = np.linalg.norm(E - c.U[:, :5], axis=0) / np.linalg.norm(c.U[:, :5], axis=0)
        assert err.max() <= 1e-5
        # a repeated transmitter: residual block of rank below its width
        pos = np.concatenate([p.src_pos[:3], p.src_pos[:1]])
        mom = np.concatenate([p.src_mom[:3], p.src_mom[:1]])
        E, _, info = c.ctx.solve(pos, mom, rtol=1e-9)
        assert info["converged"] and info["fallback"] == 4
        assert np.linalg.norm(E[:, 3] - E[:, 0]) <= 1e-9 * np.linalg.norm(E[:, 0])
        # a zero right-hand side column
        b = c.B[:, :3].copy()
        b[:, 1] = 0
        x, info = c.ctx.solve_rhs(b, rtol=1e-9)
        assert info["converged"] and info["fallback"] == 4 and np.abs(x[:, 1]).max() == 0
        # 40 columns: two groups of 20 in lockstep, each its own block space
        b40 = workload.seeded_complex((c.B.shape[0], 40), 3)
        x, info = c.ctx.solve_rhs(b40, rtol=1e-9)
        assert info["converged"] and info["fallback"] == 0
        u40 = fem.solve_direct(c.A, b40)
        err = np.linalg.norm(x - u40, axis=0) / np.linalg.norm(u40, axis=0)
        assert err.max() <= 1e-5, err
    finally:
        c.ctx.close()


def test_block_port_solve():
    print("[case] waveguide (6,3,12) ports, block FGMRES", flush=True)
    eps = 44.0 - 10.785j
    xyz, tet, pts = ports.waveguide(0.03, 0.015, 0.06, (6, 3, 12), eps)
    t = fem.Topology(xyz, tet)
    A, fp, pe = ports.assemble(t, np.full(len(tet), eps), 0, 1e9, eps, pts, pec=True)
    U = fem.solve_direct(A, ports.port_rhs(t, pts, fp, pe, 1e9))
    ctx = mx.Context(0)
    try:
        ctx.assemble(xyz, tet, np.full(len(tet), eps), mx.MX_EPS_P0, 1e9, eps)
        ctx.set_ports(pts)
        ctx.set_krylov(True)
        ctx.setup_schwarz(8, 2, precision=mx.MX_PREC_C128)
        E, S, info = ctx.solve_ports(rtol=1e-10)
        assert info["converged"] and info["fallback"] == 0
        err = np.linalg.norm(E - U, axis=0) / np.linalg.norm(U, axis=0)
        assert err.max() <= 1e-6
    finally:
        ctx.close()


def test_mode_errors():
    ctx = mx.Context(0)
    try:
        with pytest.raises(mx.MxError):
            mx._check(mx.lib().mx_set_krylov(ctx._h, 7))
    finally:
        ctx.close()
