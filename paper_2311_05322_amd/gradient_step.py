"""One quasi-Newton gradient evaluation of the inverse problem at scale
(Sec. IV-D, eq. (4)): the all-transmitter forward solve at the current
permittivity, the receiver fields, and the adjoint solve whose sources are
the weighted conjugate misfits, accumulated into the gradient with respect to
the piecewise-linear permittivity, all on one GPU.

Workload: the cylindrical chamber at a 3.16 mm lattice (2.08M edges, 2048
subdomains of about 3.2k unknowns, one vertex layer of overlap; 176 GB of
complex64 subdomain storage, where a 4M-edge chamber with 2048 subdomains
would need about 430 GB), 32 z-dipoles on a ring
of radius 0.11 m that also serve as receivers. Synthetic "measured" data come
from a solve with the injured phantom (seeded tear) on a differently jittered
mesh of the same chamber (mesh seed 1, so the inversion does not use the mesh
that made its data); the current iterate is the healthy phantom on mesh seed
0; misfit weights 1/|S_meas|^2 off the diagonal; Tikhonov weight 1e-6. Complex64 factors under FP64 block FGMRES,
with the learned coarse term when weights for the 2.08M-edge chamber exist.

The gradient is checked against central differences of the GPU cost along
two directions (the gradient itself and a complex bump centred on the tear),
the costs evaluated at relative residual 1e-10.

python -m paper_2311_05322_amd.gradient_step [--c 0.00316] [--nsub 2048] [--out FILE]
Prints one JSON line.
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

import workload  # noqa: E402
import paper_2311_05322_amd as mx  # noqa: E402


def run(c=0.00316, nsub=2048, nsrc=32, alpha=1e-6, weights=None, out=None):
    """The gradient evaluation and its finite-difference check; returns the
    summary dict (and writes the markdown summary to `out` if given)."""
    if weights is None:
        weights = os.path.join(HERE, "weights", "coarse_chamber2m.npz")
    a = argparse.Namespace(c=c, nsub=nsub, nsrc=nsrc, alpha=alpha, weights=weights, out=out)
    freq = 1e9
    eb = workload.eps_r(*workload.MATERIALS["matching"], freq)
    pos, mom = workload.dipole_ring(a.nsrc, 0.11, (0.0, 0.0), 0.10)
    t0 = time.perf_counter()
    xyz_d, tet_d = workload.jittered_cylinder(0.12, 0.2, a.c, 1)
    xyz, tet = workload.jittered_cylinder(0.12, 0.2, a.c, 0)
    injured = workload.shoulder_phantom(0)
    eps_meas = workload.eps_of_labels(injured.labels(xyz_d), freq)
    eps_cur = workload.eps_of_labels(workload.shoulder_phantom(None).labels(xyz), freq)
    t_mesh_py = time.perf_counter() - t0
    print(f"[gradient] mesh {len(xyz)} vertices {len(tet)} tetrahedra ({t_mesh_py:.1f} s)", file=sys.stderr, flush=True)

    ctx = mx.Context(0)
    ctx.set_krylov(True)
    learned = os.path.exists(a.weights)
    try:
        if learned:
            from paper_2311_05322_amd.train_coarse import load_weights

        def mesh(x, t, eps):
            ctx.assemble(x, t, eps, mx.MX_EPS_P1, freq, eb)
            ctx.setup_schwarz(a.nsub, 1, precision=mx.MX_PREC_C64, factor=False, coarse=learned)
            if learned:
                load_weights(ctx, a.weights)

        # measured data on the data mesh
        mesh(xyz_d, tet_d, eps_meas)
        ctx.setup_schwarz(a.nsub, 1, precision=mx.MX_PREC_C64, coarse=learned)
        _, S_meas, info = ctx.solve(pos, mom, rtol=1e-10, want_E=False)
        if not info["converged"]:
            raise SystemExit("data solve did not converge")
        t0 = time.perf_counter()
        mesh(xyz, tet, eps_cur)
        t_topo = time.perf_counter() - t0
        sz = ctx.sizes()
        print(f"[gradient] ne={sz.ne} nv={sz.nv} nsub={sz.nsub} (topology + partition {t_topo:.1f} s)",
              file=sys.stderr, flush=True)

        def forward(eps, rtol):
            ctx.assemble(None, None, eps, mx.MX_EPS_P1, freq, eb, reuse_mesh=True)
            ctx.setup_schwarz(a.nsub, 1, precision=mx.MX_PREC_C64, coarse=learned)
            _, S, info = ctx.solve(pos, mom, rtol=rtol, want_E=False)
            if not info["converged"]:
                raise SystemExit("forward solve did not converge")
            return S, info

        w = 1.0 / np.abs(S_meas) ** 2
        np.fill_diagonal(w, 0.0)

        def cost_grad(eps, rtol):
            t0 = time.perf_counter()
            _, finfo = forward(eps, rtol)
            t1 = time.perf_counter()
            J, g, ginfo = ctx.gradient(S_meas, w, a.alpha)
            t2 = time.perf_counter()
            if not ginfo["converged"]:
                raise SystemExit("adjoint solve did not converge")
            return J, g.copy(), {"s_forward": t1 - t0, "s_adjoint_gradient": t2 - t1,
                                 "forward_steps": int(finfo["iters_max"]), "adjoint_steps": int(ginfo["iters_max"]),
                                 "forward_relres": float(finfo["relres"].max()),
                                 "adjoint_relres": float(ginfo["relres"].max()),
                                 "t_setup": finfo["t_setup"], "t_lu": finfo["t_lu"]}

        # the timed evaluation: the bench tolerance (first call warms the
        # autotuner and the graphs; the second is reported)
        cost_grad(eps_cur, 1e-8)
        J8, g8, tim = cost_grad(eps_cur, 1e-8)
        print(f"[gradient] evaluation at rtol 1e-8: {json.dumps(tim)}", file=sys.stderr, flush=True)

        # central differences of the cost at rtol 1e-10
        J, g, _ = cost_grad(eps_cur, 1e-10)
        tc = np.asarray(injured.tear_centre, dtype=float)
        r2 = np.sum((xyz - tc) ** 2, axis=1)
        dirs = {"gradient": g / np.abs(g).max(), "tear_bump": np.exp(-r2 / (2 * 0.015 ** 2)) * (1.0 - 0.3j)}
        h = 0.01
        checks = {}
        for name, d in dirs.items():
            Jp, _, _ = cost_grad(eps_cur + h * d, 1e-10)
            Jm, _, _ = cost_grad(eps_cur - h * d, 1e-10)
            fd = (Jp - Jm) / (2 * h)
            pred = float(np.real(np.vdot(g, d)))
            checks[name] = {"fd": fd, "adjoint": pred, "rel_diff": abs(fd - pred) / abs(fd)}
            print(f"[gradient] direction {name}: {checks[name]}", file=sys.stderr, flush=True)
        gdiff = float(np.linalg.norm(g8 - g) / np.linalg.norm(g))
        out = {"ne": int(sz.ne), "nv": int(sz.nv), "nsub": int(sz.nsub), "transmitters": len(pos),
               "learned_term": learned, "J": J, "J_rtol1e-8": J8, "grad_rel_diff_rtol1e-8_vs_1e-10": gdiff,
               "s_gradient_evaluation": tim["s_forward"] + tim["s_adjoint_gradient"], **tim,
               "fd_checks": checks}
        if a.out:
            lines = ["# One gradient evaluation on the 2.08M-edge chamber (Sec. IV-D, eq. (4))", "",
                     "Command (repository root on the MI355X box):", "", "```",
                     "python3 -u -m paper_2311_05322_amd.gradient_step --out profiles/gradient_chamber2m.md", "```", "",
                     f"Mesh: {sz.ne} edges, {sz.nv} vertices, {sz.nsub} subdomains (one vertex layer of overlap), "
                     f"{len(pos)} transmitters = receivers; data from the injured phantom (tear seed 0) on a "
                     f"second mesh of the chamber (jitter seed 1), current iterate the healthy phantom on mesh "
                     f"seed 0, weights 1/|S_meas|^2 off the diagonal, alpha {a.alpha:g}; "
                     f"complex64 factors, FP64 block FGMRES, learned coarse term: {'yes' if learned else 'no'}.", "",
                     "| phase (rtol 1e-8) | value |", "|---|---:|",
                     f"| forward: operator values, local matrices, LU, 32-transmitter solve (s) | {tim['s_forward']:.2f} |",
                     f"| of which set-up / LU (s) | {tim['t_setup']:.2f} / {tim['t_lu']:.2f} |",
                     f"| adjoint 32-source solve + gradient accumulation (s) | {tim['s_adjoint_gradient']:.2f} |",
                     f"| whole gradient evaluation (s) | {out['s_gradient_evaluation']:.2f} |",
                     f"| forward / adjoint block steps | {tim['forward_steps']} / {tim['adjoint_steps']} |",
                     f"| largest true residual forward / adjoint | {tim['forward_relres']:.2e} / "
                     f"{tim['adjoint_relres']:.2e} |",
                     f"| gradient at rtol 1e-8 vs 1e-10 (relative l2) | {gdiff:.2e} |", "",
                     "Central differences of the GPU cost (rtol 1e-10, step 0.01 in permittivity units) against "
                     "Re<g, d>:", "",
                     "| direction | finite difference | adjoint gradient | relative difference |",
                     "|---|---:|---:|---:|"]
            for name, c in checks.items():
                lines.append(f"| {name} | {c['fd']:.9e} | {c['adjoint']:.9e} | {c['rel_diff']:.1e} |")
            lines.append("")
            with open(a.out, "w") as f:
                f.write("\n".join(lines))
        return out
    finally:
        ctx.close()


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--c", type=float, default=0.00316, help="lattice cube size of the chamber mesh (m)")
    ap.add_argument("--nsub", type=int, default=2048)
    ap.add_argument("--nsrc", type=int, default=32)
    ap.add_argument("--alpha", type=float, default=1e-6)
    ap.add_argument("--weights", default=None, help="learned coarse-term weights (.npz; default: the 2.08M chamber's)")
    ap.add_argument("--out", default=None, help="markdown summary file")
    a = ap.parse_args()
    print(json.dumps(run(a.c, a.nsub, a.nsrc, a.alpha, a.weights, a.out)), flush=True)


if __name__ == "__main__":
    main()
