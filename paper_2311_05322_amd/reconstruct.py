"""Quasi-Newton reconstruction of the permittivity (Sec. IV-D).

The unknown is the piecewise-linear relative permittivity of an inverse mesh
(one complex value per vertex). The cost is eq. (4): the misfit of the
scattering matrix normalised by the empty-chamber data plus the Tikhonov term
on kappa = k0^2 eps. Each cost and gradient evaluation is one all-transmitter
solve (mx_solve) and one adjoint solve with the same factors (mx_gradient),
both on the GPU; the outer iteration is limited-memory BFGS with an Armijo
backtracking line search on the vector of real and imaginary parts, which
costs O(m nv) host arithmetic per iteration next to two all-transmitter solves.

Metrics of Sec. VI, eqs. (6)-(7): err = ||Re eps_rec - Re eps_exact|| / ||Re eps_exact||
(whole domain and injury area), ctr = mean over the injury area of
eps_rec(injured data) - eps_rec(healthy data).

python -m paper_2311_05322_amd.reconstruct [--c 0.008] [--iters 10] [--healthy]
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(HERE))


def _dot(a, b):
    """Real inner product of complex vectors seen as (Re, Im) pairs."""
    return float(np.real(np.vdot(a, b)))


def lbfgs_direction(g, pairs):
    """-H g by the two-loop recursion over the stored (s, y) pairs (oldest
    first), initial Hessian scaled by s'y / y'y of the newest pair."""
    q = g.copy()
    alphas = []
    for s, y in reversed(pairs):
        rho = 1.0 / _dot(y, s)
        a = rho * _dot(s, q)
        alphas.append(a)
        q = q - a * y
    if pairs:
        s, y = pairs[-1]
        q = q * (_dot(s, y) / _dot(y, y))
    for (s, y), a in zip(pairs, reversed(alphas)):
        rho = 1.0 / _dot(y, s)
        b = rho * _dot(y, q)
        q = q + (a - b) * s
    return -q


def minimize(fg, x0, iters, memory=5, first_step=1.0, project=None, c1=1e-4, max_backtrack=12, log=None):
    """L-BFGS with Armijo backtracking. fg(x) -> (f, g); g is the gradient
    with respect to (Re x, Im x) packed as g_re + 1j g_im. The first
    direction is scaled so that its largest entry has modulus first_step.
    project(x) maps a trial point into the admissible set."""
    x = np.array(x0, dtype=np.complex128)
    f, g = fg(x)
    hist = [{"iter": 0, "f": f, "gnorm": float(np.linalg.norm(g)), "evals": 1}]
    pairs = []
    evals = 1
    for it in range(1, iters + 1):
        d = lbfgs_direction(g, pairs)
        if not pairs:
            d = d * (first_step / max(np.abs(d).max(), 1e-300))
        slope = _dot(g, d)
        if slope >= 0:  # not a descent direction: restart from steepest descent
            pairs = []
            d = -g * (first_step / max(np.abs(g).max(), 1e-300))
            slope = _dot(g, d)
        t = 1.0
        for _ in range(max_backtrack):
            xt = x + t * d
            if project is not None:
                xt = project(xt)
            ft, gt = fg(xt)
            evals += 1
            if ft <= f + c1 * t * slope:
                break
            t *= 0.5
        else:
            hist.append({"iter": it, "f": f, "gnorm": float(np.linalg.norm(g)), "evals": evals, "stalled": True})
            break
        s, y = xt - x, gt - g
        if _dot(s, y) > 1e-12 * np.sqrt(_dot(s, s) * _dot(y, y)):
            pairs.append((s, y))
            pairs = pairs[-memory:]
        x, f, g = xt, ft, gt
        hist.append({"iter": it, "f": f, "gnorm": float(np.linalg.norm(g)), "evals": evals, "step": t})
        if log:
            log(hist[-1])
    return x, hist


def run_reconstruction(c=0.008, nsub=64, nsrc=32, iters=10, alpha=1e-6, snr_db=None, tear_seed=0, healthy=False,
                       first_step=2.0, verbose=True):
    """Synthetic data from the injured phantom on the direct mesh (jitter
    seed 1, permittivity labelled at its vertices), reconstruction on the
    inverse mesh (jitter seed 0) from the homogeneous matching medium.
    Returns a dict with the cost history and the err / ctr metrics."""
    import workload
    import paper_2311_05322_amd as mx

    freq = 1e9
    eb = workload.eps_r(*workload.MATERIALS["matching"], freq)
    pos, mom = workload.dipole_ring(nsrc, 0.11, (0.0, 0.0), 0.10)
    xyz_d, tet_d = workload.jittered_cylinder(0.12, 0.2, c, 1)
    xyz_i, tet_i = workload.jittered_cylinder(0.12, 0.2, c, 0)
    ph = workload.shoulder_phantom(tear_seed)
    ctx = mx.Context(0)
    opts = dict(precision=mx.MX_PREC_C64)
    try:
        def data(xyz, tet, eps):
            ctx.assemble(xyz, tet, eps, mx.MX_EPS_P1, freq, eb)
            ctx.setup_schwarz(nsub, 1, **opts)
            _, S, info = ctx.solve(pos, mom, rtol=1e-10, want_E=False)
            return S

        rng = np.random.default_rng(12345)

        def noisy(S):
            if snr_db is None:
                return S
            sig = 10.0 ** (-snr_db / 20.0)
            return (S.real * (1 + sig * rng.standard_normal(S.shape))
                    + 1j * S.imag * (1 + sig * rng.standard_normal(S.shape)))

        S_empty = data(xyz_i, tet_i, np.full(len(xyz_i), eb))
        w = 1.0 / np.abs(S_empty) ** 2
        np.fill_diagonal(w, 0.0)
        eps_inj = workload.eps_of_labels(ph.labels(xyz_d), freq)
        eps_healthy = workload.eps_of_labels(workload.shoulder_phantom(None).labels(xyz_d), freq)
        lab_i = ph.labels(xyz_i)
        exact_i = workload.eps_of_labels(lab_i, freq)
        tear_i = lab_i == workload.LABEL_NAMES.index("tear")

        def run(S_meas, name):
            first = [True]

            def fg(eps):
                ctx.assemble(xyz_i if first[0] else None, tet_i if first[0] else None, eps, mx.MX_EPS_P1, freq, eb,
                             reuse_mesh=not first[0])
                first[0] = False
                ctx.setup_schwarz(nsub, 1, **opts)
                ctx.solve(pos, mom, rtol=1e-8, want_E=False)
                J, g, _ = ctx.gradient(S_meas, w, alpha)
                return J, g.copy()

            def project(eps):
                return np.maximum(eps.real, 1.0) + 1j * np.minimum(eps.imag, 0.0)

            t0 = time.time()

            def log(h):
                if verbose:
                    print(json.dumps({"run": name, **h, "seconds": time.time() - t0}), flush=True)

            eps, hist = minimize(fg, np.full(len(xyz_i), eb), iters, first_step=first_step, project=project, log=log)
            err = np.linalg.norm(eps.real - exact_i.real) / np.linalg.norm(exact_i.real)
            err_t = (np.linalg.norm(eps.real[tear_i] - exact_i.real[tear_i]) / np.linalg.norm(exact_i.real[tear_i])
                     if tear_i.any() else float("nan"))
            return eps, hist, err, err_t, time.time() - t0

        eps0_err = np.linalg.norm(eb.real - exact_i.real) / np.linalg.norm(exact_i.real)
        S_meas = noisy(data(xyz_d, tet_d, eps_inj))
        eps_r, hist, err, err_t, sec = run(S_meas, "injured")
        out = {"ne_inverse": int(ctx.sizes().ne), "nv_inverse": len(xyz_i), "iters": iters,
               "history": [h["f"] for h in hist], "err_start": float(eps0_err), "err": float(err),
               "err_injury": float(err_t), "injury_vertices": int(tear_i.sum()), "seconds": sec}
        if healthy:
            S_h = noisy(data(xyz_d, tet_d, eps_healthy))
            eps_h, _, _, _, _ = run(S_h, "healthy")
            if tear_i.any():
                ctr = complex(np.mean(eps_r[tear_i] - eps_h[tear_i]))
                out["ctr"] = [ctr.real, ctr.imag]
        return out
    finally:
        ctx.close()


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--c", type=float, default=0.008, help="lattice cube size of both meshes")
    ap.add_argument("--nsub", type=int, default=64)
    ap.add_argument("--nsrc", type=int, default=32)
    ap.add_argument("--iters", type=int, default=10)
    ap.add_argument("--alpha", type=float, default=1e-6)
    ap.add_argument("--snr-db", type=float, default=None, help="multiplicative noise on the data (None: none)")
    ap.add_argument("--tear-seed", type=int, default=0)
    ap.add_argument("--healthy", action="store_true", help="also reconstruct from healthy data and report ctr")
    ap.add_argument("--first-step", type=float, default=2.0)
    a = ap.parse_args()
    out = run_reconstruction(a.c, a.nsub, a.nsrc, a.iters, a.alpha, a.snr_db, a.tear_seed, a.healthy, a.first_step)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
