"""Host logic of the reconstruction loop: the L-BFGS two-loop recursion and
the Armijo line search, on problems whose minimiser is known."""
import numpy as np

from paper_2311_05322_amd.reconstruct import lbfgs_direction, minimize


def _quadratic(n=20, seed=0):
    rng = np.random.default_rng(seed)
    Q = rng.standard_normal((2 * n, 2 * n))
    H = Q @ Q.T + 2 * n * np.eye(2 * n)           # SPD Hessian of the (Re, Im) vector
    xs = rng.standard_normal(n) + 1j * rng.standard_normal(n)
    zs = np.concatenate([xs.real, xs.imag])

    def fg(x):
        z = np.concatenate([x.real, x.imag]) - zs
        gz = H @ z
        return 0.5 * z @ gz, gz[:n] + 1j * gz[n:]
    return fg, xs, H


def test_two_loop_is_inverse_hessian_on_quadratic():
    """With pairs (s, H s) spanning the space, -direction equals H^{-1} g
    in the exact-arithmetic limit of BFGS on a quadratic after n updates;
    here: for one pair the secant equation H_new y = s holds."""
    fg, xs, H = _quadratic(4)
    rng = np.random.default_rng(1)
    s = rng.standard_normal(4) + 1j * rng.standard_normal(4)
    zs = np.concatenate([s.real, s.imag])
    hy = H @ zs
    y = hy[:4] + 1j * hy[4:]
    d = lbfgs_direction(y, [(s, y)])
    assert np.allclose(-d, s)


def test_minimize_quadratic_to_tolerance():
    fg, xs, _ = _quadratic(20)
    x, hist = minimize(fg, np.zeros(20, complex), iters=200, memory=8, first_step=1.0)
    assert np.linalg.norm(x - xs) <= 1e-6 * np.linalg.norm(xs)
    f = [h["f"] for h in hist]
    assert all(b <= a for a, b in zip(f, f[1:]))


def test_minimize_respects_projection():
    """Minimiser outside the box: the projected iteration stays admissible."""
    fg, xs, _ = _quadratic(6, seed=3)
    proj = lambda x: np.maximum(x.real, 0.0) + 1j * np.minimum(x.imag, 0.0)
    x, hist = minimize(fg, np.zeros(6, complex), iters=30, project=proj)
    assert np.all(x.real >= 0) and np.all(x.imag <= 0)
    assert hist[-1]["f"] <= hist[0]["f"]
