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
    assert tun["spmm_variant"] in (0, 1, 2)
    if nrhs > 32:
        assert tun["spmm_variant"] != 1


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


@pytest.mark.parametrize("prec", [0, 1])
def test_every_kernel_variant_same_answer(chamber, prec):
    """Every SpMM variant, triangular-solve order and right-hand-side width
    per workgroup gives the same solution (to the solve tolerance) and the
    direct solution."""
    p, t, A, ctx = chamber
    ctx.setup_schwarz(p.nsub, p.overlap, precision=prec)
    B = workload.seeded_complex((t.ne, 20), 19)
    U = fem.solve_direct(A, B)
    ref = None
    try:
        for spmm in (0, 1, 2):
            for paired in (0, 1):
                for cols in (16, 32):
                    print(f"[case] precision {prec} spmm {spmm} paired {paired} cols {cols}", flush=True)
                    ctx.set_tuning(spmm, paired, cols)
                    X, info = ctx.solve_rhs(B, rtol=1e-10)
                    assert info["converged"]
                    err = np.linalg.norm(X - U, axis=0) / np.linalg.norm(U, axis=0)
                    assert err.max() <= (1e-6 if prec == 0 else 1e-5)
                    if ref is None:
                        ref = X
                    assert np.linalg.norm(X - ref) <= 1e-8 * np.linalg.norm(ref)
    finally:
        ctx.set_autotune(True)


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


def _fan(k):
    """k tetrahedra around one axis edge: that edge's row of the operator has
    3k + 1 non-zeros (axis, 2k spokes, k rim edges)."""
    ang = 2 * np.pi * np.arange(k) / k
    xyz = np.concatenate([[[0.0, 0.0, -0.05], [0.0, 0.0, 0.05]],
                          np.stack([0.04 * np.cos(ang), 0.04 * np.sin(ang), np.zeros(k)], 1)])
    tet = np.array([[0, 1, 2 + i, 2 + (i + 1) % k] for i in range(k)], np.int32)
    return xyz, tet


@pytest.mark.parametrize("k", [16, 50])
def test_spmm_long_rows(k):
    """A row longer than two 16-entry chunks (49 non-zeros) goes through the
    column-window SpMM's tail loop; a row longer than a window (151 > 128
    columns) leaves that variant unavailable (MX_EINVAL when asked for) and
    every other variant still matches A @ X."""
    print(f"[case] spmm fan of {k} tetrahedra", flush=True)
    xyz, tet = _fan(k)
    eps = np.full(len(tet), workload.eps_r(44.0, 0.6, 1e9))
    t = fem.Topology(xyz, tet)
    assert np.diff(t.row_ptr).max() == 3 * k + 1
    A = fem.assemble(t, eps, 0, 1e9, eps[0])
    X = workload.seeded_complex((t.ne, 20), 3)
    ref = A @ X
    ctx = mx.Context(0)
    try:
        ctx.assemble(xyz, tet, eps, 0, 1e9, eps[0])
        variants = (0, 1, 2) if 3 * k + 1 <= 128 else (0, 1)
        if 3 * k + 1 > 128:
            with pytest.raises(mx.MxError) as e:
                ctx.set_tuning(2, 1, 32)
            assert e.value.code == mx.MX_EINVAL
        for v in variants:
            ctx.set_tuning(v, 1, 32)
            Y = ctx.apply_operator(X)
            assert np.abs(Y - ref).max() <= 1e-13 * np.abs(ref).max(), v
    finally:
        ctx.close()


def test_mesh_errors_and_orientation():
    """A zero-volume tetrahedron and a frequency that is not positive are
    MX_EINVAL; a tetrahedron given with the opposite orientation (two vertex
    ids swapped) yields bitwise the same operator values."""
    print("[case] edges: degenerate / inverted tetrahedra, k0 = 0", flush=True)
    xyz, tet = workload.kuhn_cube(3, 0.1)
    eps = np.full(len(tet), workload.eps_r(44.0, 0.6, 1e9))
    ctx = mx.Context(0)
    try:
        ctx.assemble(xyz, tet, eps, 0, 1e9, eps[0])
        v_ref = ctx.matrix_values()
        flipped = tet.copy()
        flipped[::2, [0, 1]] = flipped[::2, [1, 0]]          # every other tet inverted
        ctx.assemble(xyz, flipped, eps, 0, 1e9, eps[0])
        assert np.array_equal(ctx.matrix_values(), v_ref)
        bad = tet.copy()
        bad[5] = [bad[5][0], bad[5][1], bad[5][2], bad[5][2]]  # repeated vertex
        with pytest.raises(mx.MxError) as e:
            ctx.assemble(xyz, bad, eps, 0, 1e9, eps[0])
        assert e.value.code == mx.MX_EINVAL
        flat = xyz.copy()
        flat[:, 2] = 0.0                                      # every tetrahedron has zero volume
        with pytest.raises(mx.MxError) as e:
            ctx.assemble(flat, tet, eps, 0, 1e9, eps[0])
        assert e.value.code == mx.MX_EINVAL
        for f in (0.0, -1e9, float("nan")):
            with pytest.raises(mx.MxError) as e:
                ctx.assemble(xyz, tet, eps, 0, f, eps[0])
            assert e.value.code == mx.MX_EINVAL
    finally:
        ctx.close()


def test_pivot_error_and_timings():
    """Complex64 factors of a permittivity whose mass term exceeds the
    complex64 range: the first pivot is infinite, the elimination turns the
    next column into non-finite values and the factorisation reports
    MX_EPIVOT; a solve afterwards is MX_ESTATE. A normal set-up then reports
    its assembly, set-up and factorisation times in the solve diagnostics."""
    print("[case] edges: MX_EPIVOT on complex64 overflow", flush=True)
    xyz, tet = workload.kuhn_cube(4, 0.1)
    ctx = mx.Context(0)
    try:
        huge = np.full(len(tet), 1e50 + 0j)   # k0^2 eps |T| / 120 ~ 1e43 > FLT_MAX
        ctx.assemble(xyz, tet, huge, 0, 1e9, 44.0)
        with pytest.raises(mx.MxError) as e:
            ctx.setup_schwarz(8, 1, precision=mx.MX_PREC_C64)
        assert e.value.code == mx.MX_EPIVOT
        with pytest.raises(mx.MxError) as e:
            ctx.solve_rhs(np.ones((ctx.ne, 1), np.complex128))
        assert e.value.code == mx.MX_ESTATE
        eps = np.full(len(tet), workload.eps_r(44.0, 0.6, 1e9))
        ctx.assemble(xyz, tet, eps, 0, 1e9, eps[0])
        ctx.setup_schwarz(8, 1, precision=mx.MX_PREC_C64)
        _, info = ctx.solve_rhs(workload.seeded_complex((ctx.ne, 2), 3), rtol=1e-8)
        assert info["converged"]
        assert info["t_assemble"] > 0 and info["t_setup"] > 0 and 0 < info["t_lu"] <= info["t_setup"]
    finally:
        ctx.close()


def test_context_on_caller_stream():
    """A context created on a caller stream (torch's) runs there and gives
    the same answer as one on its own stream."""
    torch = pytest.importorskip("torch")
    print("[case] edges: context on a torch stream", flush=True)
    p = workload.cube_problem(n=5, nsub=8, overlap=1, nsrc=3)
    st = torch.cuda.Stream()
    outs = []
    for stream in (None, st.cuda_stream):
        ctx = mx.Context(0, stream=stream)
        try:
            # same kernel variants in both contexts (the autotuner's timing
            # could pick different ones, which agree only to rounding)
            ctx.set_tuning(1, 1, 32)
            ctx.set_lu_group(2)
            ctx.assemble(p.xyz, p.tet, p.eps, p.eps_kind, p.freq, p.eps_b)
            ctx.setup_schwarz(p.nsub, p.overlap)
            E, S, info = ctx.solve(p.src_pos, p.src_mom, rtol=1e-10)
            assert info["converged"]
            outs.append(E)
        finally:
            ctx.close()
    assert np.array_equal(outs[0], outs[1])


def test_tuning_cache(tmp_path, monkeypatch):
    """With MX_TUNE_CACHE set, the first context times the variants and the
    panel groups and stores its picks; a second context on the same problem
    takes them from the file without timing and computes bitwise the same
    fields (same kernels in the same order)."""
    import json
    path = tmp_path / "tune.json"
    monkeypatch.setenv("MX_TUNE_CACHE", str(path))
    print("[case] edges: tuning cache c=30mm nsub=8", flush=True)
    p = workload.chamber_problem(c=0.03, nsub=8, overlap=1, nsrc=4)
    outs = []
    for _ in range(2):
        ctx = mx.Context(0)
        try:
            ctx.assemble(p.xyz, p.tet, p.eps, p.eps_kind, p.freq, p.eps_b)
            ctx.setup_schwarz(p.nsub, p.overlap, precision=mx.MX_PREC_C64)
            E, S, info = ctx.solve(p.src_pos, p.src_mom, rtol=1e-10)
            assert info["converged"]
            outs.append((E, ctx.tuning()))
        finally:
            ctx.close()
    (E0, t0), (E1, t1) = outs
    print(t0, t1, flush=True)
    assert t0["from_cache"] == {"solve": False, "lu": False}
    assert min(t0["lu_ms_groups_1_2_4_8"]) > 0
    assert t1["from_cache"] == {"solve": True, "lu": True}
    assert t1["lu_ms_groups_1_2_4_8"] == [0.0] * 4
    for k in ("spmm_variant", "trsm_paired", "trsm_cols", "lu_group"):
        assert t1[k] == t0[k], k
    assert np.array_equal(E0, E1)
    data = json.loads(path.read_text())
    lu = [v for k, v in data.items() if k.startswith("lu:1:8:")]
    sv = [v for k, v in data.items() if k.startswith("solve:")]
    assert len(lu) == 1 and lu[0] == {"group": t0["lu_group"]}
    assert len(sv) == 1 and sv[0] == {"spmm": t0["spmm_variant"], "trsm_paired": t0["trsm_paired"],
                                      "trsm_cols": t0["trsm_cols"]}
