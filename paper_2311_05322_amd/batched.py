"""Batched form: several phantoms, each with many transmitters, solved one
after another on one GPU.

Each phantom has its own seeded mesh (0.6M-1.4M edges), tear and number of
subdomains (uneven subdomains of about 2.5k-5.5k unknowns), and 160 unit
z-dipoles on 5 rings of 32 at z = 0.06 ... 0.14 m, adjacent rings rotated by
half a pitch (the shifted rings of the paper's antenna study, Sec. VI). One
all-transmitter solve per phantom: operator values, local matrices and the
banded LU of all subdomains, block FGMRES of all 160 transmitters (five
groups of 32 advancing in lockstep, one preconditioner and operator
application over the whole width) to relative residual 1e-8, complex64
factors under the FP64 iteration. The mesh topology and the partition of a
phantom are built before its solve and timed apart (they do not depend on the
permittivity). The phantoms are staged: one context holds one phantom's
factors and Krylov space at a time (the largest needs about 0.24 TB).

python -m paper_2311_05322_amd.batched [--phantoms 8] [--rings 5] [--tune-cache FILE] [--out profiles/batched_c3.md]
Prints one JSON line per phantom and a summary line.
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


def solve_phantom(ctx, p, restart, want_E=False, rtol=None):
    """One phantom of the batch on a context in block mode: topology and
    partition (timed apart), then operator values, local matrices, LU and
    the all-transmitter block FGMRES solve. Returns (E or None, info,
    seconds of topology + partition, seconds of the solve)."""
    t0 = time.perf_counter()
    ctx.assemble(p.xyz, p.tet, p.eps, p.eps_kind, p.freq, p.eps_b)
    ctx.setup_schwarz(p.nsub, p.overlap, precision=mx.MX_PREC_C64, factor=False, restart=restart)
    t_mesh = time.perf_counter() - t0
    t0 = time.perf_counter()
    ctx.assemble(None, None, p.eps, p.eps_kind, p.freq, p.eps_b, reuse_mesh=True)
    ctx.setup_schwarz(p.nsub, p.overlap, precision=mx.MX_PREC_C64, restart=restart)
    E, _, info = ctx.solve(p.src_pos, p.src_mom, rtol=rtol or p.rtol, want_E=want_E)
    return (E if want_E else None), info, t_mesh, time.perf_counter() - t0


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--phantoms", type=int, default=8)
    ap.add_argument("--rings", type=int, default=5)
    ap.add_argument("--per-ring", type=int, default=32)
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--restart", type=int, default=10,
                    help="restart length in block steps (10 keeps the 160-column Krylov space of the largest "
                         "phantom near 0.08 TB)")
    ap.add_argument("--out", default=None, help="markdown summary file")
    ap.add_argument("--tune-cache", default=None,
                    help="autotuning cache file (MX_TUNE_CACHE): picks found there are not timed again")
    a = ap.parse_args()
    if a.tune_cache:
        os.environ["MX_TUNE_CACHE"] = a.tune_cache
    warm = bool(a.tune_cache) and os.path.exists(a.tune_cache)
    specs = workload.batched_specs(a.phantoms, a.seed)
    ctx = mx.Context(0)
    ctx.set_krylov(True)
    rows = []
    t_all = 0.0
    try:
        for k, sp in enumerate(specs):
            p = workload.chamber_problem(c=sp["c"], mesh_seed=sp["mesh_seed"], tear_seed=sp["tear_seed"],
                                         nsub=sp["nsub"], overlap=1, nsrc=a.per_ring, rings=a.rings)
            print(f"[phantom {k}] c={sp['c'] * 1000:.2f} mm nsub={sp['nsub']} transmitters={len(p.src_pos)}",
                  file=sys.stderr, flush=True)
            _, info, t_mesh, t_solve = solve_phantom(ctx, p, a.restart)
            t_all += t_solve
            sz = ctx.sizes()
            _, dp, *_ = ctx.partition()
            ni = [int(dp[i + 1] - dp[i]) for i in range(sz.nsub)]
            row = {"phantom": k, "c_mm": sp["c"] * 1000, "ne": int(sz.ne), "nsub": int(sz.nsub),
                   "n_i_min": min(ni), "n_i_max": max(ni), "transmitters": len(p.src_pos),
                   "block_steps": int(info["iters_max"]), "converged": bool(info["converged"]),
                   "max_relres": float(info["relres"].max()), "s_topology_partition": t_mesh,
                   "s_solve": t_solve, "s_setup": info["t_setup"], "s_lu": info["t_lu"], "s_iter": info["t_iter"],
                   "lu_tiles": int(sz.lu_tiles)}
            rows.append(row)
            print(json.dumps(row), flush=True)
            if not info["converged"]:
                raise SystemExit(f"phantom {k} did not converge")
    finally:
        ctx.close()
    ntx = sum(r["transmitters"] for r in rows)
    summary = {"phantoms": len(rows), "transmitter_solves": ntx, "s_solves_total": t_all,
               "phantom_solves_per_s": len(rows) / t_all, "transmitter_solves_per_s": ntx / t_all,
               "ne_range": [min(r["ne"] for r in rows), max(r["ne"] for r in rows)],
               "n_i_range": [min(r["n_i_min"] for r in rows), max(r["n_i_max"] for r in rows)]}
    print(json.dumps(summary), flush=True)
    if a.out:
        lines = ["# Batched form: 8 phantoms x 160 transmitters, staged through one MI355X", "",
                 "Command (repository root on the MI355X box):", "", "```",
                 "python3 -u -m paper_2311_05322_amd.batched " + " ".join(sys.argv[1:]), "```", "",
                 "Per phantom: own seeded mesh and tear, 5 shifted rings x 32 z-dipoles, complex64 banded LU, "
                 "block FGMRES (groups of 32 in lockstep), rtol 1e-8 (true residual). `solve` = operator values + "
                 "local matrices + LU + iterations; topology and partition are built before it and timed apart. "
                 + ("Tuning cache: " + ("warm (picks read from the file, nothing timed)" if warm else
                                         "cold (the autotuner times each new shape bucket inside that phantom's solve)")
                    if a.tune_cache else
                    "No tuning cache: the autotuner times each new shape bucket inside that phantom's solve."),
                 "",
                 "| phantom | c (mm) | edges | subdomains | n_i | block steps | max relres | topology+partition s | "
                 "solve s | of which LU s | iterations s |",
                 "|---:|---:|---:|---:|---|---:|---:|---:|---:|---:|---:|"]
        for r in rows:
            lines.append(f"| {r['phantom']} | {r['c_mm']:.2f} | {r['ne']} | {r['nsub']} | {r['n_i_min']}-{r['n_i_max']} | "
                         f"{r['block_steps']} | {r['max_relres']:.2e} | {r['s_topology_partition']:.1f} | "
                         f"{r['s_solve']:.2f} | {r['s_lu']:.2f} | {r['s_iter']:.2f} |")
        lines += ["", f"Total: {len(rows)} phantoms, {ntx} transmitter solves in {t_all:.1f} s of solves: "
                  f"{summary['phantom_solves_per_s']:.3f} phantom solves/s, "
                  f"{summary['transmitter_solves_per_s']:.1f} transmitter solves/s.", ""]
        with open(a.out, "w") as f:
            f.write("\n".join(lines))


if __name__ == "__main__":
    main()
