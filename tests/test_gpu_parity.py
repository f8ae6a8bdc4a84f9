"""GPU path (through the C ABI) against the CPU oracle on seeded inputs.

Integer maps (edges, tetrahedron->edge map, CSR pattern, partition, DOF
lists, partition-of-unity weights, colours) must match bit for bit; the
assembled operator to rounding; one ORAS application to 1e-10 (complex128
factors) / 1e-5 (complex64); solved fields to relative l2 1e-6 (FP64 path)
and 1e-5 (mixed path), the criteria of the solver's accuracy targets.
"""
import numpy as np
import pytest

import workload
from oracle import fem, krylov, schwarz

mx = pytest.importorskip("paper_2311_05322_amd")
pytestmark = pytest.mark.gpu


def _case(name, **kw):
    if name == "cube8":
        return workload.cube_problem(n=8, **kw)
    if name == "chamber20":
        return workload.chamber_problem(c=0.02, nsub=16, overlap=2, nsrc=8, **kw)
    raise KeyError(name)


class Case:
    def __init__(self, name):
        print(f"[case] {name}", flush=True)
        self.p = p = _case(name)
        self.t = fem.Topology(p.xyz, p.tet)
        self.A = fem.assemble(self.t, p.eps, p.eps_kind, p.freq, p.eps_b)
        self.ctx = mx.Context(0)
        self.ctx.assemble(p.xyz, p.tet, p.eps, p.eps_kind, p.freq, p.eps_b)


@pytest.fixture(scope="module", params=["cube8", "chamber20"])
def case(request):
    c = Case(request.param)
    yield c
    c.ctx.close()


def test_topology_bit_exact(case):
    edges, t2e, rp, col = case.ctx.topology()
    assert np.array_equal(edges, case.t.edges)
    assert np.array_equal(t2e, case.t.t2e)
    assert np.array_equal(rp, case.t.row_ptr)
    assert np.array_equal(col, case.t.col)


def test_operator_values(case):
    v = case.ctx.matrix_values()
    ref = case.A.data
    assert np.abs(v - ref).max() <= 1e-13 * np.abs(ref).max()


@pytest.mark.parametrize("variant", [0, 1, 2])
def test_spmm(case, variant):
    """Every SpMM variant against A @ X: 32 right-hand sides, a ragged count
    (5) and 20 (the column-window variant's second block half full)."""
    X = workload.seeded_complex((case.t.ne, 32), 7)
    ref = case.A @ X
    case.ctx.set_tuning(variant, 1, 32)
    try:
        for n in (32, 5, 20):
            Xn = np.ascontiguousarray(X[:, :n])
            Yn = case.ctx.apply_operator(Xn)
            assert np.abs(Yn - ref[:, :n]).max() <= 1e-13 * np.abs(ref).max(), n
    finally:
        case.ctx.set_autotune(True)


@pytest.mark.parametrize("overlap", [1, 2])
def test_partition_bit_exact(case, overlap):
    p = case.p
    case.ctx.setup_schwarz(p.nsub, overlap, factor=False)
    dec = schwarz.Decomposition(case.t, p.nsub, overlap)
    part, dp, dofs, w, col = case.ctx.partition()
    assert np.array_equal(part, dec.part)
    assert np.array_equal(dp, dec.dof_ptr)
    assert np.array_equal(dofs, np.concatenate(dec.dofs))
    assert np.array_equal(w, np.concatenate(dec.w))
    assert np.array_equal(col, dec.colour)


def test_local_matrices(case):
    p = case.p
    case.ctx.setup_schwarz(p.nsub, p.overlap, factor=False)
    dec = schwarz.Decomposition(case.t, p.nsub, p.overlap)
    for i in sorted({0, p.nsub // 2, p.nsub - 1}):
        B = case.ctx.local_matrix(i)
        ref = dec.local_matrix(i, p.eps, p.eps_kind, p.freq, p.eps_b).toarray()
        assert np.abs(B - ref).max() <= 1e-13 * np.abs(ref).max(), i


@pytest.mark.parametrize("prec,tol", [(0, 1e-10), (1, 2e-5)])
def test_preconditioner_application(case, prec, tol):
    p = case.p
    case.ctx.setup_schwarz(p.nsub, p.overlap, precision=prec)
    dec = schwarz.Decomposition(case.t, p.nsub, p.overlap)
    M = schwarz.ORAS(dec, p.eps, p.eps_kind, p.freq, p.eps_b, dense=True)
    X = workload.seeded_complex((case.t.ne, 8), 11)
    Z = case.ctx.apply_preconditioner(X)
    ref = M.apply(X)
    err = np.linalg.norm(Z - ref, axis=0) / np.linalg.norm(ref, axis=0)
    assert err.max() <= tol, err


@pytest.mark.parametrize("prec,tol", [(0, 1e-10), (1, 2e-5)])
def test_preconditioner_every_panel_group(case, prec, tol):
    """The factorisation's panels per trailing-update pass (the autotuner's
    choice) changes only the rounding: one ORAS application per group
    against the oracle's."""
    p = case.p
    dec = schwarz.Decomposition(case.t, p.nsub, p.overlap)
    M = schwarz.ORAS(dec, p.eps, p.eps_kind, p.freq, p.eps_b, dense=True)
    X = workload.seeded_complex((case.t.ne, 8), 12)
    ref = M.apply(X)
    try:
        for g in (1, 3, 4, 8, 16):
            case.ctx.set_lu_group(g)
            case.ctx.setup_schwarz(p.nsub, p.overlap, precision=prec)
            Z = case.ctx.apply_preconditioner(X)
            err = np.linalg.norm(Z - ref, axis=0) / np.linalg.norm(ref, axis=0)
            print("group", g, "err", err.max(), flush=True)
            assert err.max() <= tol, (g, err)
    finally:
        case.ctx.set_lu_group(0)


@pytest.mark.parametrize("prec", [0, 1])
def test_setup_after_factorisation(case, prec):
    """A set-up that follows a completed factorisation clears only the factor
    tiles inside that factorisation's recorded extents before it gathers the
    new local matrices. A factorisation of another permittivity in between
    must leave no trace: the preconditioner of the original permittivity
    comes out bit for bit as before, and the dense local matrices of a later
    unfactored set-up equal the oracle's entry by entry."""
    p = case.p
    X = workload.seeded_complex((case.t.ne, 8), 13)
    case.ctx.set_tuning(1, 1, 32)
    try:
        case.ctx.setup_schwarz(p.nsub, p.overlap, precision=prec)
        Z1 = case.ctx.apply_preconditioner(X)
        case.ctx.assemble(None, None, p.eps * (1.7 - 0.4j), p.eps_kind, p.freq, p.eps_b, reuse_mesh=True)
        case.ctx.setup_schwarz(p.nsub, p.overlap, precision=prec)
        Zo = case.ctx.apply_preconditioner(X)
        assert not np.array_equal(Zo, Z1)
        case.ctx.assemble(None, None, p.eps, p.eps_kind, p.freq, p.eps_b, reuse_mesh=True)
        case.ctx.setup_schwarz(p.nsub, p.overlap, precision=prec)
        Z2 = case.ctx.apply_preconditioner(X)
        assert np.array_equal(Z1, Z2)
        case.ctx.setup_schwarz(p.nsub, p.overlap, precision=prec, factor=False)
        dec = schwarz.Decomposition(case.t, p.nsub, p.overlap)
        tol = 1e-13 if prec == 0 else 2.0 ** -23  # complex64 storage: one rounding per entry
        for i in range(p.nsub):
            B = case.ctx.local_matrix(i)
            ref = dec.local_matrix(i, p.eps, p.eps_kind, p.freq, p.eps_b).toarray()
            assert np.all(np.abs(B - ref) <= tol * np.abs(ref) + 1e-13 * np.abs(ref).max()), i
    finally:
        case.ctx.set_autotune(True)


@pytest.mark.parametrize("prec,tol", [(0, 1e-6), (1, 1e-5)])
def test_fields_match_direct_solve(case, prec, tol):
    p = case.p
    case.ctx.setup_schwarz(p.nsub, p.overlap, precision=prec)
    E, S, info = case.ctx.solve(p.src_pos, p.src_mom, rtol=1e-10)
    assert info["converged"] and np.all(info["relres"] <= 1e-10)
    B = fem.dipole_rhs(case.t, p.src_pos, p.src_mom, p.freq)
    U = fem.solve_direct(case.A, B)
    err = np.linalg.norm(E - U, axis=0) / np.linalg.norm(U, axis=0)
    print("iters", info["iters"], "field err", err.max())
    assert err.max() <= tol
    R = fem.functionals(case.t, p.src_pos, p.src_mom)
    Sref = fem.scattering(R, U)
    assert np.abs(S - Sref).max() <= tol * np.abs(Sref).max()
    assert np.abs(S - S.T).max() <= 10 * tol * np.abs(S).max()
    # true residual re-checked with the oracle's operator
    res = np.linalg.norm(B - case.A @ E, axis=0) / np.linalg.norm(B, axis=0)
    assert res.max() <= 1e-9


def test_iteration_counts_close_to_oracle(case):
    p = case.p
    case.ctx.setup_schwarz(p.nsub, p.overlap, precision=0, restart=40)
    _, _, info = case.ctx.solve(p.src_pos[:2], p.src_mom[:2], rtol=1e-8, want_E=False)
    dec = schwarz.Decomposition(case.t, p.nsub, p.overlap)
    M = schwarz.ORAS(dec, p.eps, p.eps_kind, p.freq, p.eps_b)
    B = fem.dipole_rhs(case.t, p.src_pos[:2], p.src_mom[:2], p.freq)
    _, its, _ = krylov.fgmres_block(case.A, M.apply, B, 1e-8, 40)
    print("gpu iters", info["iters"], "oracle iters", its)
    assert np.all(np.abs(info["iters"] - its) <= 2)


def test_point_functionals(case):
    p = case.p
    R = case.ctx.point_functionals(p.src_pos, p.src_mom)
    ref = fem.functionals(case.t, p.src_pos, p.src_mom)
    assert np.abs(R - ref).max() <= 1e-12 * np.abs(ref).max()
    assert np.array_equal(R != 0, ref != 0)


def test_manufactured_solution(case):
    p = case.p
    case.ctx.setup_schwarz(p.nsub, p.overlap, precision=1)
    u = workload.seeded_complex((case.t.ne, 3), 5)
    b = case.A @ u
    x, info = case.ctx.solve_rhs(b, rtol=1e-10)
    assert info["converged"]
    assert (np.linalg.norm(x - u, axis=0) / np.linalg.norm(u, axis=0)).max() < 1e-6


# -- single-subdomain and error paths (cube only) ---------------------------

@pytest.fixture(scope="module")
def cube():
    c = Case("cube8")
    yield c
    c.ctx.close()


def test_one_subdomain_converges_in_one_step(cube):
    p = cube.p
    cube.ctx.setup_schwarz(1, 1, precision=0)
    _, _, info = cube.ctx.solve(p.src_pos[:4], p.src_mom[:4], rtol=1e-8, want_E=False)
    assert info["converged"] and info["iters_max"] == 1


def test_errors(cube):
    p = cube.p
    c = mx.Context(0)
    with pytest.raises(mx.MxError) as e:
        c.setup_schwarz(8, 1)
    assert e.value.code == mx.MX_ESTATE
    bad = p.eps.copy()
    bad[3] = np.nan
    with pytest.raises(mx.MxError) as e:
        c.assemble(p.xyz, p.tet, bad, 0, p.freq, p.eps_b)
    assert e.value.code == mx.MX_EINVAL
    c.assemble(p.xyz, p.tet, p.eps, 0, p.freq, p.eps_b)
    with pytest.raises(mx.MxError) as e:
        c.setup_schwarz(6, 1)
    assert e.value.code == mx.MX_EINVAL
    c.setup_schwarz(8, 1, maxit=1)
    _, _, info = c.solve(p.src_pos[:2], p.src_mom[:2], rtol=1e-8, want_E=False)
    assert not info["converged"]
    with pytest.raises(mx.MxError) as e:
        c.solve(np.array([[0.5, 0.5, 0.5]]), np.array([[0, 0, 1]]), rtol=1e-8)
    assert e.value.code == mx.MX_EINVAL
    c.close()
