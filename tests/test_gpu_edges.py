"""Edge cases of the solve through the C ABI against the oracle's direct
solve: right-hand-side counts that are not multiples of the 32-wide tiles
(1, 5, 33, 40: partial column tiles of the triangular solves, the SpMM and
Gram-Schmidt variants for more than 32 right-hand sides, the autotuner and
the graph cache re-keyed per count), a zero right-hand side, and the
autotuner switched off."""
import numpy as np
import pytest

import workload
from oracle import fem

mx = pytest.importorskip("paper_2311_05322_amd")
pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def chamber():
    print("[case] edges chamber c=20mm nsub=16 overlap=1", flush=True)
    p = workload.chamber_problem(c=0.02, nsub=16, overlap=1, nsrc=8)
    t = fem.Topology(p.xyz, p.tet)
    A = fem.assemble(t, p.eps, p.eps_kind, p.freq, p.eps_b)
    ctx = mx.Context(0)
    ctx.assemble(p.xyz, p.tet, p.eps, p.eps_kind, p.freq, p.eps_b)
    yield p, t, A, ctx
    ctx.close()


@pytest.mark.parametrize("nrhs", [1, 5, 33, 40])
@pytest.mark.parametrize("prec,tol", [(0, 1e-6), (1, 1e-5)])
def test_ragged_rhs_counts(chamber, nrhs, prec, tol):
    p, t, A, ctx = chamber
    ctx.setup_schwarz(p.nsub, p.overlap, precision=prec)
    B = workload.seeded_complex((t.ne, nrhs), 100 + nrhs)
    for rep in range(2):  # second pass: tuned variants and captured graphs
        X, info = ctx.solve_rhs(B, rtol=1e-10)
        assert info["converged"], (nrhs, rep)
        U = fem.solve_direct(A, B)
        err = np.linalg.norm(X - U, axis=0) / np.linalg.norm(U, axis=0)
        assert err.max() <= tol, (nrhs, rep, err.max())
    tun = ctx.tuning()
    assert tun["spmm_variant"] in (0, 1)
    if nrhs > 32:
        assert tun["spmm_variant"] == 0


def test_zero_rhs_column(chamber):
    """A zero column converges at once to zero; the others are unaffected."""
    p, t, A, ctx = chamber
    ctx.setup_schwarz(p.nsub, p.overlap, precision=1)
    B = workload.seeded_complex((t.ne, 4), 7)
    B[:, 2] = 0
    X, info = ctx.solve_rhs(B, rtol=1e-10)
    assert info["converged"]
    assert np.all(X[:, 2] == 0)
    U = fem.solve_direct(A, B[:, [0, 1, 3]])
    err = np.linalg.norm(X[:, [0, 1, 3]] - U, axis=0) / np.linalg.norm(U, axis=0)
    assert err.max() <= 1e-5


def test_autotune_off_same_answer(chamber):
    p, t, A, ctx = chamber
    ctx.setup_schwarz(p.nsub, p.overlap, precision=1)
    B = workload.seeded_complex((t.ne, 8), 9)
    X1, _ = ctx.solve_rhs(B, rtol=1e-10)
    ctx.set_autotune(False)
    try:
        X2, info = ctx.solve_rhs(B, rtol=1e-10)
        assert info["converged"]
        assert ctx.tuning()["spmm_variant"] == 0
    finally:
        ctx.set_autotune(True)
    assert np.linalg.norm(X1 - X2) <= 1e-8 * np.linalg.norm(X1)


def test_limits_are_errors():
    """Sizes beyond the documented limits are rejected before any launch:
    a subdomain above 8192 unknowns, more than 256 right-hand sides, no
    transmitters."""
    xyz, tet = workload.kuhn_cube(14, 0.1)   # 18,389 edges in one subdomain
    ctx = mx.Context(0)
    try:
        eps = np.full(len(tet), workload.eps_r(44.0, 0.6, 1e9))
        ctx.assemble(xyz, tet, eps, 0, 1e9, eps[0])
        with pytest.raises(mx.MxError) as e:
            ctx.setup_schwarz(1, 1)
        assert e.value.code == mx.MX_EINVAL
        ctx.setup_schwarz(8, 1)
        B = np.zeros((ctx.ne, 257), np.complex128)
        with pytest.raises(mx.MxError) as e:
            ctx.solve_rhs(B)
        assert e.value.code == mx.MX_EINVAL
        with pytest.raises(mx.MxError) as e:
            ctx.solve(np.zeros((0, 3)), np.zeros((0, 3)), rtol=1e-8)
        assert e.value.code == mx.MX_EINVAL
    finally:
        ctx.close()
