"""Time of one all-transmitter solve against the number of antennas.

The transmitters are N unit z-dipoles on the ring r = 0.11 m (z = 0.10 m) of
the 1.02M-edge chamber; every N is one block right-hand side. One step is the
same as in bench.py: operator values, dense ORAS matrices + batched LU, block
FGMRES of all N transmitters to relative residual 1e-8. The sweep mirrors the
paper's study of run time against antenna count (Sec. VI, Table II) on the
synthetic phantom; the reconstruction-quality columns of that table need the
paper's shoulder model and are not reproduced.

python -m paper_2311_05322_amd.antenna_sweep [--counts 16,32,64,96] [--steps 2] [--krylov block]
Prints one JSON line per count and a markdown table at the end.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(HERE))

import workload  # noqa: E402
import paper_2311_05322_amd as mx  # noqa: E402


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--counts", default="16,32,64,96")
    ap.add_argument("--steps", type=int, default=2)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--c", type=float, default=0.004, help="lattice cube size (4 mm: 1.02M edges)")
    ap.add_argument("--nsub", type=int, default=512)
    ap.add_argument("--precision", choices=["c64", "c128"], default="c64")
    ap.add_argument("--krylov", choices=["pseudo", "block"], default="pseudo",
                    help="pseudo-block FGMRES or block FGMRES (groups of at most 32 transmitters)")
    a = ap.parse_args()
    prec = mx.MX_PREC_C64 if a.precision == "c64" else mx.MX_PREC_C128
    ctx = mx.Context(0)
    ctx.set_krylov(a.krylov == "block")
    rows = []
    first = True
    for n in (int(x) for x in a.counts.split(",")):
        p = workload.chamber_problem(c=a.c, nsub=a.nsub, overlap=1, nsrc=n)
        if first:
            ctx.assemble(p.xyz, p.tet, p.eps, p.eps_kind, p.freq, p.eps_b)
            first = False

        def step():
            ctx.assemble(None, None, p.eps, p.eps_kind, p.freq, p.eps_b, reuse_mesh=True)
            ctx.setup_schwarz(p.nsub, p.overlap, precision=prec)
            _, _, info = ctx.solve(p.src_pos, p.src_mom, rtol=p.rtol, want_E=False)
            return info

        for _ in range(a.warmup):
            step()
        t0 = time.perf_counter()
        infos = [step() for _ in range(a.steps)]
        dt = (time.perf_counter() - t0) / a.steps
        row = {"antennas": n, "s_per_solve": dt, "s_per_transmitter": dt / n,
               "iters": int(infos[-1]["iters_max"]), "converged": bool(infos[-1]["converged"]),
               "precision": a.precision, "krylov": a.krylov, "ne": int(ctx.sizes().ne), "nsub": a.nsub}
        rows.append(row)
        print(json.dumps(row), flush=True)
    ctx.close()
    print("| antennas | s per all-transmitter solve | s per transmitter | iterations |")
    print("|---:|---:|---:|---:|")
    for r in rows:
        print(f"| {r['antennas']} | {r['s_per_solve']:.2f} | {r['s_per_transmitter']:.3f} | {r['iters']} |")


if __name__ == "__main__":
    main()
