"""Pins of the oracle's adjoint gradient: central finite differences of the
cost (each J from direct solves) and the P1 stiffness on linear fields."""
import numpy as np
import pytest

import workload
from oracle import fem, gradient


def p1_problem(n=4, seed=0):
    xyz, tet = workload.kuhn_cube(n, 0.1)
    t = fem.Topology(xyz, tet)
    rng = np.random.default_rng(seed)
    eb = workload.eps_r(44.0, 0.6, 1e9)
    eps = eb + 3.0 * rng.standard_normal(t.nv) - 1.0j * np.abs(rng.standard_normal(t.nv))
    pos, mom = workload.dipole_ring(4, 0.03, (0.05, 0.05), 0.047)
    return t, eps, eb, pos, mom


def test_p1_stiffness_kills_linear_fields():
    xyz, tet = workload.kuhn_cube(4)
    t = fem.Topology(xyz, tet)
    K1 = gradient.p1_stiffness(t)
    lin = 2.0 + 3.0 * t.xyz[:, 0] - 1.5 * t.xyz[:, 1] + 0.7 * t.xyz[:, 2]
    r = K1 @ lin
    interior = np.all((t.xyz > 1e-9) & (t.xyz < 0.1 - 1e-9), axis=1)
    assert np.abs(r[interior]).max() < 1e-12 * np.abs(K1).max()
    assert np.abs(K1 @ np.ones(t.nv)).max() < 1e-12 * np.abs(K1).max()


@pytest.mark.parametrize("alpha", [0.0, 1e-6])
def test_gradient_matches_finite_differences(alpha):
    t, eps, eb, pos, mom = p1_problem()
    # "measured" data from a perturbed permittivity
    rng = np.random.default_rng(3)
    eps_true = eps + 2.0 * rng.standard_normal(t.nv)
    _, (_, _, _, S_meas, _) = gradient.misfit(t, eps_true, 1e9, eb, pos, mom, np.zeros((4, 4)), np.ones((4, 4)))
    w = 1.0 / np.abs(S_meas) ** 2
    np.fill_diagonal(w, 0.0)
    J, g, _ = gradient.gradient(t, eps, 1e9, eb, pos, mom, S_meas, w, alpha)
    for k in range(3):
        dvec = rng.standard_normal(t.nv) + 1j * rng.standard_normal(t.nv)
        h = 1e-4
        Jp = gradient.cost(t, eps + h * dvec, 1e9, eb, pos, mom, S_meas, w, alpha)
        Jm = gradient.cost(t, eps - h * dvec, 1e9, eb, pos, mom, S_meas, w, alpha)
        fd = (Jp - Jm) / (2 * h)
        an = np.real(np.vdot(g, dvec))
        assert abs(fd - an) <= 1e-6 * abs(fd) + 1e-14 * abs(J), (fd, an)
