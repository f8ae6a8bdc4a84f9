"""All-port solves of the waveguide-port chamber model on one GPU.

The antennas are open-ended ceramic-filled waveguides (eps_r = 59, TE10,
Sec. III and IV-B): rectangular apertures on the side walls of a box chamber
with metallic walls elsewhere, the shoulder phantom inside and the matching
liquid around it. Every port transmits in turn (g = 2 j beta e_TE10 on its
aperture, all ports as one block right-hand side) and every port receives
(eq. (3)). One step: operator values with the port and wall conditions,
dense ORAS subdomain matrices + batched LU, block FGMRES of all ports to
relative residual 1e-8, scattering matrix.

python -m paper_2311_05322_amd.port_chamber [--h 0.0042] [--ports-per-wall 4]
    [--precision c64,c64-block,c128] [--steps 2]
Prints one JSON line per precision (progress on stderr).
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


def box_problem(h=0.0042, ports_per_wall=4, rings=(0.4, 0.6), freq=1e9, tear_seed=0):
    """Mesh, P0 permittivity, background permittivity and ports of the
    0.24 x 0.24 x 0.2 m box chamber at lattice size h (4.2 mm: 1.16M edges)."""
    xyz, tet, pts = workload.box_chamber(0.24, 0.2, h, ports_per_wall, rings)
    lab = workload.shoulder_phantom(tear_seed).labels(workload.tet_centroids(xyz, tet))
    eps = workload.eps_of_labels(lab, freq)
    eb = workload.eps_r(*workload.MATERIALS["matching"], freq)
    return xyz, tet, eps, eb, pts


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--h", type=float, default=0.0042, help="lattice cube size (4.2 mm: 1.16M edges)")
    ap.add_argument("--ports-per-wall", type=int, default=4, help="apertures per wall and ring (two rings)")
    ap.add_argument("--nsub", type=int, default=512)
    ap.add_argument("--overlap", type=int, default=1)
    ap.add_argument("--precision", default="c64,c128",
                    help="comma-separated runs: c64, c128, or c64-block (block FGMRES, complex64 factors)")
    ap.add_argument("--rtol", type=float, default=1e-8)
    ap.add_argument("--steps", type=int, default=2)
    ap.add_argument("--warmup", type=int, default=1)
    a = ap.parse_args()
    freq = 1e9
    xyz, tet, eps, eb, pts = box_problem(a.h, a.ports_per_wall, freq=freq)
    ctx = mx.Context(0)
    try:
        t = time.perf_counter()
        ctx.assemble(xyz, tet, eps, mx.MX_EPS_P0, freq, eb)
        ctx.set_ports(pts, pec=True)
        print(f"mesh + ports: {time.perf_counter() - t:.1f} s, ne={ctx.sizes().ne}, ports={len(pts)}",
              file=sys.stderr, flush=True)
        for name in a.precision.split(","):
            prec = mx.MX_PREC_C128 if name == "c128" else mx.MX_PREC_C64
            ctx.set_krylov(name.endswith("-block"))

            def step():
                ctx.assemble(None, None, eps, mx.MX_EPS_P0, freq, eb, reuse_mesh=True)
                ctx.setup_schwarz(a.nsub, a.overlap, precision=prec)
                _, S, info = ctx.solve_ports(rtol=a.rtol, want_E=False)
                return S, info

            for w in range(a.warmup):
                _, info = step()
                print(f"{name} warmup {w}: iters {info['iters_max']}", file=sys.stderr, flush=True)
            t0 = time.perf_counter()  # solve_ports returns after the stream has drained
            for k in range(a.steps):
                S, info = step()
                print(f"{name} step {k}: iters {info['iters_max']} relres {info['relres'].max():.2e}",
                      file=sys.stderr, flush=True)
            dt = (time.perf_counter() - t0) / a.steps
            ctx.set_profiling(True)
            step()
            kt = ctx.kernel_times()
            ctx.set_profiling(False)
            sz = ctx.sizes()
            row = {"workload": f"box chamber h={a.h * 1000:g} mm", "precision": name, "ne": int(sz.ne),
                   "nsub": int(sz.nsub), "overlap": a.overlap, "ports": len(pts), "rtol": a.rtol,
                   "s_per_solve": dt, "solves_per_s": 1.0 / dt, "iters": int(info["iters_max"]),
                   "converged": bool(info["converged"]), "relres_max": float(info["relres"].max()),
                   "reciprocity": float(np.abs(S - S.T).max() / np.abs(S).max()),
                   "S_diag_abs_mean": float(np.abs(np.diag(S)).mean()),
                   "kernel_ms_per_step": {k: v[0] for k, v in kt.items() if v[1]}}
            print(json.dumps(row), flush=True)
    finally:
        ctx.close()


if __name__ == "__main__":
    main()
