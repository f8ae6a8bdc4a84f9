"""Pins of the learned-coarse-space oracle: lattice prolongation exact on
linear fields, bf16 rounding, network backward vs finite differences, and
least-squares targets that reproduce a coarse-representable error."""
import numpy as np
import pytest

import workload
from oracle import fem, learned, schwarz


@pytest.fixture(scope="module")
def small():
    p = workload.cube_problem(n=6, nsub=8, overlap=1)
    t = fem.Topology(p.xyz, p.tet)
    dec = schwarz.Decomposition(t, 8, 1)
    return p, t, dec


def test_prolongation_reproduces_linear_fields(small):
    """Trilinear hats sum to one and reproduce linear functions, so nodal
    values of E(x) = a + B x give the exact edge circulations."""
    p, t, dec = small
    rng = np.random.default_rng(0)
    a = rng.standard_normal(3)
    B = rng.standard_normal((3, 3))
    for i in (0, 5):
        lo, hi = learned.subdomain_box(t, dec.tets[i])
        P = learned.lattice_prolongation(t, dec.dofs[i], lo, hi)
        g = np.linspace(0, 1, 4)
        c = np.zeros(learned.NCOARSE)
        for cc in range(4):
            for bb in range(4):
                for aa in range(4):
                    x = lo + (hi - lo) * np.array([g[aa], g[bb], g[cc]])
                    node = aa + 4 * bb + 16 * cc
                    c[3 * node:3 * node + 3] = a + B @ x
        xa = t.xyz[t.edges[dec.dofs[i], 0]]
        xb = t.xyz[t.edges[dec.dofs[i], 1]]
        mid = 0.5 * (xa + xb)
        exact = ((a[None] + mid @ B.T) * (xb - xa)).sum(1)     # midpoint rule is exact for linear E
        assert np.abs(P @ c - exact).max() < 1e-13 * np.abs(exact).max()


def test_bf16_rounding():
    """Round-to-nearest-even on the top 16 bits of a float32."""
    vals = np.array([1.0, 1.0 + 2 ** -8, 1.0 + 2 ** -7, 1.0 + 3 * 2 ** -8, -2.5, 3.14159, 1e-30], np.float32)
    got = learned.bf16(vals)
    # 1 + 2^-8 is a tie between 1 and 1 + 2^-7 -> even (1); 1 + 3*2^-8 ties -> 1 + 2^-6
    assert got[0] == 1.0 and got[1] == 1.0 and got[2] == 1.0 + 2 ** -7 and got[3] == 1.0 + 2 ** -6
    assert got[4] == -2.5
    assert abs(got[5] - 3.140625) < 1e-12
    rel = np.abs(got - vals) / np.abs(vals)
    assert np.all(rel <= 2 ** -8)


def test_backward_matches_finite_differences(small):
    p, t, dec = small
    nb = [dec.neighbours(i) for i in range(dec.nsub)]
    rng = np.random.default_rng(1)
    theta = learned.init_params(3, out_scale=1.0)
    X = rng.standard_normal((2, dec.nsub, learned.NIN))
    Y = rng.standard_normal((2, dec.nsub, learned.NIN))
    L, g = learned.loss_and_grad(theta, X, Y, nb, use_bf16=False)
    for _ in range(4):
        d = rng.standard_normal(theta.size)
        h = 1e-5
        Lp, _ = learned.loss_and_grad(theta + h * d, X, Y, nb, use_bf16=False)
        Lm, _ = learned.loss_and_grad(theta - h * d, X, Y, nb, use_bf16=False)
        fd = (Lp - Lm) / (2 * h)
        assert abs(fd - g @ d) <= 1e-6 * abs(fd) + 1e-12
    # neighbour mean and its adjoint
    a = rng.standard_normal((1, dec.nsub, 5))
    b = rng.standard_normal((1, dec.nsub, 5))
    assert abs(np.sum(learned.neighbour_mean(a, nb) * b) - np.sum(a * learned.neighbour_mean_T(b, nb))) < 1e-12


def test_targets_recover_coarse_error(small):
    """If e - M^{-1} r restricted to every subdomain is exactly P_i c, the
    least-squares target returns c (up to the small ridge)."""
    p, t, dec = small
    co = learned.Coarse(dec)
    rng = np.random.default_rng(2)
    # a global linear field a + B x interpolated on the edges is P_i c_i on every subdomain
    a = rng.standard_normal(3)
    B = rng.standard_normal((3, 3))
    xa = t.xyz[t.edges[:, 0]]
    xb = t.xyz[t.edges[:, 1]]
    u = ((a[None] + (0.5 * (xa + xb)) @ B.T) * (xb - xa)).sum(1)[:, None].astype(np.complex128)
    r = np.ones_like(u)                      # s = 1
    c = co.targets(r, u, np.zeros_like(u))
    for i in range(dec.nsub):
        rec = co.P[i] @ (c[0, i, :192] + 1j * c[0, i, 192:])
        sw = np.sqrt(dec.D[i])
        ui = u[dec.dofs[i], 0]
        # the fit is exact up to the ridge, measured in the D-weighted norm it minimises
        assert np.linalg.norm(sw * (rec - ui)) <= 1e-4 * np.linalg.norm(sw * ui)
    q = co.correction(c, r)
    assert np.linalg.norm(q[:, 0] - u[:, 0]) <= 1e-4 * np.linalg.norm(u)


def test_theta_combination_is_the_least_squares_weight():
    """theta_j minimises ||v_j - A(z1_j + theta q_j)||: the residual it leaves is
    orthogonal to A q_j, never exceeds that of theta = 0, and any perturbed
    weight does worse; a zero correction gets theta = 0."""
    rng = np.random.default_rng(21)
    n = 60
    A = rng.standard_normal((n, n)) + 1j * rng.standard_normal((n, n)) + 8 * np.eye(n)
    v = rng.standard_normal((n, 3)) + 1j * rng.standard_normal((n, 3))
    z1 = np.linalg.solve(A + 0.3 * rng.standard_normal((n, n)), v)
    q = rng.standard_normal((n, 3)) + 1j * rng.standard_normal((n, 3))
    q[:, 2] = 0
    z, th = learned.theta_combination(A, v, z1, q)
    assert th[2] == 0 and np.array_equal(z[:, 2], z1[:, 2])
    res = v - A @ z
    for j in range(2):
        aq = A @ q[:, j]
        assert abs(np.vdot(aq, res[:, j])) <= 1e-12 * np.linalg.norm(aq) * np.linalg.norm(res[:, j])
        r0 = np.linalg.norm(v[:, j] - A @ z1[:, j])
        r1 = np.linalg.norm(res[:, j])
        assert r1 <= r0
        for d in (1e-3, -1e-3, 1e-3j, -1e-3j):
            assert np.linalg.norm(v[:, j] - A @ (z1[:, j] + (th[j] + d) * q[:, j])) > r1
