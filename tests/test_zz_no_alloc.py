"""mx_apply_preconditioner_noalloc against mx_apply_preconditioner through
the C ABI: the same one-level ORAS application with the restricted vectors in
the library's fixed device array instead of context-allocated memory. Two calls
in a row (the second with fewer right-hand sides, so the array keeps the first
call's contents beyond what the second writes), both factor precisions, and
the documented errors (too many right-hand sides for the array, host
pointers, the learned term set up)."""
import ctypes as ct

import numpy as np
import pytest

import workload

mx = pytest.importorskip("paper_2311_05322_amd")
torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def chamber():
    print("[case] no-alloc preconditioner: chamber c=20mm nsub=16 overlap=1", flush=True)
    p = workload.chamber_problem(c=0.02, nsub=16, overlap=1, nsrc=8)
    ctx = mx.Context(0)
    ctx.assemble(p.xyz, p.tet, p.eps, p.eps_kind, p.freq, p.eps_b)
    yield p, ctx
    ctx.close()


@pytest.mark.parametrize("prec,tol", [(mx.MX_PREC_C128, 1e-12), (mx.MX_PREC_C64, 1e-6)])
def test_noalloc_matches_allocating_entry_point(chamber, prec, tol):
    p, ctx = chamber
    ctx.setup_schwarz(p.nsub, p.overlap, precision=prec)
    ne = ctx.ne
    for nrhs, seed in ((7, 41), (2, 42)):
        print(f"[case] precision {prec} nrhs {nrhs}", flush=True)
        V = workload.seeded_complex((ne, nrhs), seed)
        ref = ctx.apply_preconditioner(V)
        X = torch.from_numpy(V).to("cuda")
        Z = torch.full_like(X, float("nan"))
        ctx.apply_preconditioner_noalloc(X, Z)
        torch.cuda.synchronize()
        got = Z.cpu().numpy()
        assert np.all(np.isfinite(got))
        err = np.linalg.norm(got - ref, axis=0) / np.linalg.norm(ref, axis=0)
        print("max relative difference", err.max(), "bitwise", np.array_equal(got, ref), flush=True)
        assert err.max() <= tol
        # in place (X == Z)
        ctx.apply_preconditioner_noalloc(X, X)
        torch.cuda.synchronize()
        assert np.linalg.norm(X.cpu().numpy() - got) <= tol * np.linalg.norm(ref)


def test_noalloc_errors(chamber):
    p, ctx = chamber
    ctx.setup_schwarz(p.nsub, p.overlap, precision=mx.MX_PREC_C128)
    L = mx.lib()
    V = np.zeros((ctx.ne, 2), np.complex128)
    rc = L.mx_apply_preconditioner_noalloc(ctx._h, ct.c_void_p(V.ctypes.data), ct.c_void_p(V.ctypes.data), 2)
    assert rc == mx.MX_EINVAL                      # host pointers
    X = torch.zeros((ctx.ne, 2), dtype=torch.complex128, device="cuda")
    ctx.setup_schwarz(p.nsub, p.overlap, precision=mx.MX_PREC_C128, coarse=True)
    ctx.coarse_init(seed=1)
    with pytest.raises(mx.MxError) as e:
        ctx.apply_preconditioner_noalloc(X, X)
    assert e.value.code == mx.MX_ESTATE
    ctx.setup_schwarz(p.nsub, p.overlap, precision=mx.MX_PREC_C128)


def test_noalloc_rejects_sizes_beyond_the_array():
    print("[case] no-alloc size limit: chamber c=12mm nsub=64", flush=True)
    p = workload.chamber_problem(c=0.012, nsub=64, overlap=1, nsrc=2)
    ctx = mx.Context(0)
    try:
        ctx.assemble(p.xyz, p.tet, p.eps, p.eps_kind, p.freq, p.eps_b)
        ctx.setup_schwarz(64, 1, precision=mx.MX_PREC_C128)
        s = ctx.sizes()
        dp = ctx.partition()[1]
        rows = 0
        for i in range(s.nsub):
            n = int(dp[i + 1] - dp[i])
            rows += (n + s.nb - 1) // s.nb * s.nb
        per_rhs = 16 * rows
        too_many = (64 << 20) // per_rhs + 1
        assert too_many <= 256
        X = torch.zeros((ctx.ne, too_many), dtype=torch.complex128, device="cuda")
        with pytest.raises(mx.MxError) as e:
            ctx.apply_preconditioner_noalloc(X, X)
        assert e.value.code == mx.MX_EINVAL
        ok = torch.zeros((ctx.ne, too_many - 1), dtype=torch.complex128, device="cuda")
        ctx.apply_preconditioner_noalloc(ok, ok)
        torch.cuda.synchronize()
    finally:
        ctx.close()
