"""Adjoint gradient on the GPU (through the C ABI) against the oracle's
adjoint gradient and against central finite differences of the GPU cost."""
import numpy as np
import pytest

import workload
from oracle import fem, gradient

mx = pytest.importorskip("paper_2311_05322_amd")
pytestmark = pytest.mark.gpu


def p1_case(n=6, seed=0):
    xyz, tet = workload.kuhn_cube(n, 0.1)
    t = fem.Topology(xyz, tet)
    rng = np.random.default_rng(seed)
    eb = workload.eps_r(44.0, 0.6, 1e9)
    eps = eb + 3.0 * rng.standard_normal(t.nv) - 1.0j * np.abs(rng.standard_normal(t.nv))
    pos, mom = workload.dipole_ring(6, 0.03, (0.05, 0.05), 0.047)
    eps_true = eps + 2.0 * rng.standard_normal(t.nv)
    _, (_, _, _, S_meas, _) = gradient.misfit(t, eps_true, 1e9, eb, pos, mom, 0, 1)
    w = 1.0 / np.abs(S_meas) ** 2
    np.fill_diagonal(w, 0.0)
    return xyz, tet, t, eps, eb, pos, mom, S_meas, w


def gpu_cost_grad(ctx, xyz, tet, eps, eb, pos, mom, S_meas, w, alpha, prec, first=False):
    ctx.assemble(xyz, tet, eps, mx.MX_EPS_P1, 1e9, eb, reuse_mesh=not first)
    ctx.setup_schwarz(8, 1, precision=prec)
    _, S, info = ctx.solve(pos, mom, rtol=1e-11, want_E=False)
    assert info["converged"]
    J, g, ainfo = ctx.gradient(S_meas, w, alpha)
    assert ainfo["converged"]
    return J, g, S


@pytest.mark.parametrize("prec,tol,block", [(0, 1e-6, False), (1, 1e-5, False), (0, 1e-6, True)],
                         ids=["c128", "c64", "c128-blockfgmres"])
def test_gradient_matches_oracle(prec, tol, block):
    xyz, tet, t, eps, eb, pos, mom, S_meas, w = p1_case()
    ctx = mx.Context(0)
    ctx.set_krylov(block)  # forward and adjoint solves with block FGMRES
    alpha = 1e-6
    J, g, S = gpu_cost_grad(ctx, xyz, tet, eps, eb, pos, mom, S_meas, w, alpha, prec, first=True)
    Jr, gr, Sr = gradient.gradient(t, eps, 1e9, eb, pos, mom, S_meas, w, alpha)
    assert abs(J - Jr) <= tol * abs(Jr)
    assert np.linalg.norm(g - gr) <= tol * np.linalg.norm(gr)
    ctx.close()


def test_gradient_finite_differences_of_gpu_cost():
    xyz, tet, t, eps, eb, pos, mom, S_meas, w = p1_case(n=5, seed=2)
    ctx = mx.Context(0)
    alpha = 1e-6
    J, g, _ = gpu_cost_grad(ctx, xyz, tet, eps, eb, pos, mom, S_meas, w, alpha, 0, first=True)
    rng = np.random.default_rng(9)
    for _ in range(2):
        d = rng.standard_normal(t.nv) + 1j * rng.standard_normal(t.nv)
        h = 1e-4
        Jp, _, _ = gpu_cost_grad(ctx, xyz, tet, eps + h * d, eb, pos, mom, S_meas, w, alpha, 0)
        Jm, _, _ = gpu_cost_grad(ctx, xyz, tet, eps - h * d, eb, pos, mom, S_meas, w, alpha, 0)
        fd = (Jp - Jm) / (2 * h)
        assert abs(fd - np.real(np.vdot(g, d))) <= 1e-5 * abs(fd)
    ctx.close()


def test_gradient_needs_a_solve():
    xyz, tet, t, eps, eb, pos, mom, S_meas, w = p1_case(n=4)
    ctx = mx.Context(0)
    ctx.assemble(xyz, tet, eps, mx.MX_EPS_P1, 1e9, eb)
    ctx.setup_schwarz(8, 1)
    with pytest.raises(mx.MxError) as e:
        ctx.gradient(S_meas, w, 1e-6)
    assert e.value.code == mx.MX_ESTATE
    ctx.close()


def test_gradient_step_module_small_chamber():
    """The at-scale gradient driver (forward + adjoint solves with complex64
    factors, block FGMRES and the learned term) on a 0.13M-edge chamber: its
    adjoint gradient matches central differences of the GPU cost along the
    gradient and along a bump at the tear."""
    from paper_2311_05322_amd.gradient_step import run
    print("[case] gradient_step c=8mm nsub=64", flush=True)
    out = run(c=0.008, nsub=64)
    print(out, flush=True)
    assert out["forward_relres"] <= 1e-8 and out["adjoint_relres"] <= 1e-8
    for name, c in out["fd_checks"].items():
        assert c["rel_diff"] <= 1e-5, (name, c)
