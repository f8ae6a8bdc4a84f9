"""The reconstruction loop (L-BFGS over the GPU cost and adjoint gradient)
on a small chamber: every accepted step lowers the cost of eq. (4)."""
import numpy as np
import pytest

mx = pytest.importorskip("paper_2311_05322_amd")
from paper_2311_05322_amd.reconstruct import run_reconstruction  # noqa: E402

pytestmark = pytest.mark.gpu


def test_reconstruction_lowers_cost():
    print("[case] reconstruction c=20mm nsub=16 nsrc=8 iters=3", flush=True)
    out = run_reconstruction(c=0.02, nsub=16, nsrc=8, iters=3, verbose=False)
    h = out["history"]
    print(out)
    assert len(h) >= 2 and np.all(np.isfinite(h))
    assert all(b < a for a, b in zip(h, h[1:]))
    assert h[-1] < 0.9 * h[0]


def test_reconstruction_matches_oracle_driven_loop():
    """The same L-BFGS loop (three iterations, same data, weights, start and
    projection) driven once by the GPU cost and adjoint gradient and once by
    the oracle's (direct solves): every accepted cost and the final iterate
    agree to 1e-6 (the GPU solves to rtol 1e-10 with complex128 factors)."""
    import workload
    from oracle import fem, gradient
    from paper_2311_05322_amd.reconstruct import minimize

    print("[case] reconstruction parity c=30mm nsub=8 nsrc=8 iters=3", flush=True)
    freq, alpha = 1e9, 1e-6
    eb = workload.eps_r(*workload.MATERIALS["matching"], freq)
    pos, mom = workload.dipole_ring(8, 0.11, (0.0, 0.0), 0.10)
    xyz, tet = workload.jittered_cylinder(0.12, 0.2, 0.03, 0)
    topo = fem.Topology(xyz, tet)
    ph = workload.shoulder_phantom(0)
    eps_true = workload.eps_of_labels(ph.labels(xyz), freq)
    # data and empty-chamber weights from the oracle's direct solves
    _, (_, _, _, S_empty, _) = gradient.misfit(topo, np.full(len(xyz), eb), freq, eb, pos, mom,
                                               np.zeros((8, 8), complex), np.ones((8, 8)))
    _, (_, _, _, S_meas, _) = gradient.misfit(topo, eps_true, freq, eb, pos, mom, np.zeros((8, 8), complex),
                                              np.ones((8, 8)))
    w = 1.0 / np.abs(S_empty) ** 2
    np.fill_diagonal(w, 0.0)

    def project(eps):
        return np.maximum(eps.real, 1.0) + 1j * np.minimum(eps.imag, 0.0)

    ctx = mx.Context(0)
    try:
        def fg_gpu(eps):
            ctx.assemble(xyz, tet, eps, mx.MX_EPS_P1, freq, eb)
            ctx.setup_schwarz(8, 1, precision=mx.MX_PREC_C128)
            ctx.solve(pos, mom, rtol=1e-10, want_E=False)
            J, g, info = ctx.gradient(S_meas, w, alpha)
            assert info["converged"]
            return J, g.copy()

        def fg_oracle(eps):
            J, g, _ = gradient.gradient(topo, eps, freq, eb, pos, mom, S_meas, w, alpha)
            return J, g

        x0 = np.full(len(xyz), eb)
        xg, hg = minimize(fg_gpu, x0, 3, first_step=2.0, project=project)
        xo, ho = minimize(fg_oracle, x0, 3, first_step=2.0, project=project)
    finally:
        ctx.close()
    print("gpu costs", [h["f"] for h in hg], "oracle costs", [h["f"] for h in ho], flush=True)
    assert len(hg) == len(ho) == 4
    for a, b in zip(hg, ho):
        assert abs(a["f"] - b["f"]) <= 1e-6 * abs(b["f"])
        assert a["evals"] == b["evals"]
    assert np.linalg.norm(xg - xo) <= 1e-6 * np.linalg.norm(xo)
    assert hg[-1]["f"] < 0.9 * hg[0]["f"]
