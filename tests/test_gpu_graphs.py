"""Arnoldi steps replayed from captured HIP graphs give bitwise the same
solves as eager launches: several solves in a row (each replaying the graphs
of the previous ones, with the library's own eager work and synchronisations
between the replays), a short restart so that steps recur inside one solve,
and a re-assembly with new permittivity values between solves."""
import numpy as np
import pytest

import workload

mx = pytest.importorskip("paper_2311_05322_amd")
pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("name", ["cube8", "chamber20"])
@pytest.mark.parametrize("prec", [0, 1])
def test_graph_replay_matches_eager(name, prec):
    print(f"[case] graphs {name} precision {prec}", flush=True)
    if name == "cube8":
        p = workload.cube_problem(n=8)
    else:
        p = workload.chamber_problem(c=0.02, nsub=16, overlap=1, nsrc=8)
    ctx = mx.Context(0)
    try:
        ctx.assemble(p.xyz, p.tet, p.eps, p.eps_kind, p.freq, p.eps_b)
        eps2 = p.eps * (1.0 + 0.01j)
        ref = []
        ctx.set_graphs(False)
        for e in (p.eps, eps2):
            ctx.assemble(None, None, e, p.eps_kind, p.freq, p.eps_b, reuse_mesh=True)
            ctx.setup_schwarz(p.nsub, p.overlap, precision=prec, restart=5)
            E, S, info = ctx.solve(p.src_pos, p.src_mom, rtol=1e-10)
            assert info["converged"] and info["cycles"] >= 2
            ref.append((E, info["iters"]))
        ctx.set_graphs(True)
        for rep in range(3):
            for (E0, it0), e in zip(ref, (p.eps, eps2)):
                ctx.assemble(None, None, e, p.eps_kind, p.freq, p.eps_b, reuse_mesh=True)
                ctx.setup_schwarz(p.nsub, p.overlap, precision=prec, restart=5)
                E, S, info = ctx.solve(p.src_pos, p.src_mom, rtol=1e-10)
                assert np.array_equal(info["iters"], it0), rep
                assert np.array_equal(E, E0), rep
    finally:
        ctx.close()
