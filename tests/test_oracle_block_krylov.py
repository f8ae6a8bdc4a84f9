"""Pins of the block FGMRES oracle against what the mathematics fixes:
one right-hand side is ordinary FGMRES; the block Krylov space contains
every column's own Krylov space, so with a fixed preconditioner and no
restart no column's residual after k block steps exceeds its single-vector
GMRES residual after k steps; the block space of an n x n system with s
right-hand sides is the whole space after ceil(n/s) steps; and the solution
is the direct solve's."""
import numpy as np
import pytest

import workload
from oracle import block_krylov, fem, krylov, schwarz


@pytest.fixture(scope="module")
def cube():
    p = workload.cube_problem(n=8)
    t = fem.Topology(p.xyz, p.tet)
    A = fem.assemble(t, p.eps, 0, p.freq, p.eps_b)
    dec = schwarz.Decomposition(t, 8, 1)
    M = schwarz.ORAS(dec, p.eps, 0, p.freq, p.eps_b)
    B = fem.dipole_rhs(t, p.src_pos, p.src_mom, p.freq)
    return A, M, B


def _random_system(n, seed):
    rng = np.random.default_rng(seed)
    A = rng.standard_normal((n, n)) + 1j * rng.standard_normal((n, n)) + 2.0 * n ** 0.5 * np.eye(n)
    return A


def test_one_column_is_fgmres(cube):
    A, M, B = cube
    b = B[:, 2]
    x1, it1, rr1, h1 = krylov.fgmres(lambda v: A @ v, M.apply, b, 1e-9, 30)
    X, it, rr, h = block_krylov.block_fgmres(lambda V: A @ V, M.apply, b[:, None], 1e-9, 30)
    assert it == it1
    assert np.linalg.norm(X[:, 0] - x1) <= 1e-10 * np.linalg.norm(x1)
    assert np.allclose(h, h1, rtol=1e-6, atol=1e-14)


def test_block_residuals_never_exceed_single_vector_gmres():
    n, s, k = 60, 4, 8
    A = _random_system(n, 1)
    rng = np.random.default_rng(2)
    B = rng.standard_normal((n, s)) + 1j * rng.standard_normal((n, s))
    d = 1.0 / np.diag(A)
    M = lambda V: d[:, None] * V if V.ndim == 2 else d * V      # fixed diagonal preconditioner
    _, _, _, hb = block_krylov.block_fgmres(lambda V: A @ V, M, B, 1e-30, restart=k, maxit=k)
    # the block estimate is the max over columns of the relative residual;
    # single-vector FGMRES with the same k steps on every column
    single = []
    for j in range(s):
        _, _, _, h = krylov.fgmres(lambda v: A @ v, M, B[:, j], 1e-30, restart=k, maxit=k)
        single.append(h)
    single = np.array(single)                                    # [s, k]
    for step in range(k):
        assert hb[step] <= single[:, step].max() * (1 + 1e-8)


def test_block_space_fills_in_n_over_s_steps():
    n, s = 24, 4
    A = _random_system(n, 3)
    rng = np.random.default_rng(4)
    B = rng.standard_normal((n, s)) + 1j * rng.standard_normal((n, s))
    X, it, rr, _ = block_krylov.block_fgmres(lambda V: A @ V, lambda V: V, B, 1e-11, restart=10)
    assert it <= n // s
    assert rr.max() <= 1e-10
    assert np.linalg.norm(X - np.linalg.solve(A, B)) <= 1e-9 * np.linalg.norm(X)


def test_matches_direct_solve_and_not_more_steps(cube):
    A, M, B = cube
    U = fem.solve_direct(A, B)
    X, it, rr, _ = block_krylov.block_fgmres(lambda V: A @ V, M.apply, B, 1e-9, 30)
    assert rr.max() <= 1e-9
    err = np.linalg.norm(X - U, axis=0) / np.linalg.norm(U, axis=0)
    assert err.max() <= 1e-7
    its = [krylov.fgmres(lambda v: A @ v, M.apply, B[:, j], 1e-9, 30)[1] for j in range(B.shape[1])]
    assert it <= max(its)


def test_rank_deficient_block_is_reported():
    n = 20
    A = _random_system(n, 5)
    b = np.arange(n, dtype=np.complex128) + 1.0
    with pytest.raises(block_krylov.RankDeficient):
        block_krylov.block_fgmres(lambda V: A @ V, lambda V: V, np.stack([b, 2 * b], axis=1))
    with pytest.raises(block_krylov.RankDeficient):
        block_krylov.block_fgmres(lambda V: A @ V, lambda V: V, np.stack([b, 0 * b], axis=1))
