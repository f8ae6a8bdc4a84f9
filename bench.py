#!/usr/bin/env python3
"""All-transmitter Maxwell solves per second on one MI355X.

One step = one all-transmitter solve for one permittivity map: operator
values (topology cached), dense ORAS subdomain matrices + batched LU, and
block FGMRES of every transmitter to relative residual 1e-8 (true residual
checked).  The headline variant uses complex64 subdomain factors on the
matrix cores under an FP64 outer iteration; the plain FP64 one-level Schwarz
solver is timed in the same run as the reference, and so is block FGMRES (one
Krylov space for all transmitters, variant c64_block).

python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload chamber1m|cube8]
Prints one JSON line on stdout (progress goes to stderr).
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
MFMA_PEAK_TFLOPS = {"fp32": 157.3, "fp64": 78.6}

WORKLOADS = {
    # 1.02M-edge cylindrical chamber, shoulder phantom, 32 z-dipoles on r=0.11 m,
    # 512 subdomains of about 5.2k unknowns (one vertex layer of overlap)
    "chamber1m": dict(kind="chamber", c=0.004, mesh_seed=0, tear_seed=0, nsub=512, overlap=1, nsrc=32),
    # 2.08M-edge chamber (3.16 mm lattice), 2048 subdomains of about 3.2k unknowns
    # (one vertex layer of overlap): complex64 factors 176 GB; complex128 would not fit
    "chamber2m": dict(kind="chamber", c=0.00316, mesh_seed=0, tear_seed=0, nsub=2048, overlap=1, nsrc=32),
    # same chamber family at 8 mm lattice (about 0.13M edges), 64 subdomains
    "chamber130k": dict(kind="chamber", c=0.008, mesh_seed=0, tear_seed=0, nsub=64, overlap=1, nsrc=32),
    # 4,184-edge unit cube, 8 dipoles, 8 subdomains, one layer of overlap
    "cube8": dict(kind="cube", n=8, seed=0, nsub=8, overlap=1),
}


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def make_problem(name):
    import workload
    w = dict(WORKLOADS[name])
    if w.pop("kind") == "cube":
        return workload.cube_problem(**w)
    return workload.chamber_problem(**w)


def algorithmic_work(kind, n_i, nnz, ne, nrhs, elem_bytes, kt):
    """Algorithmic flops and bytes of one launch of a kernel class, from the
    problem sizes (real subdomain sizes n_i, not the padded ones)."""
    n = n_i.astype(np.float64)
    if kind == "lu_update":
        # A22 -= L21 U12 for every 64-column panel: 8 * 64 * (n - 64(p+1))^2
        tot = 0.0
        for ni in n_i:
            m = np.arange(64, int(ni), 64, dtype=np.float64)
            tot += 8.0 * 64.0 * ((ni - m) ** 2).sum()
        nfact = max(1, kt["lu_inv"][1] // 2)          # two timed intervals per factorisation
        per = tot / max(1.0, kt["lu_update"][1] / nfact)
        return per, None
    if kind in ("trsm_lower", "trsm_upper"):
        return 4.0 * (n * n).sum() * nrhs, 0.5 * (n * n).sum() * elem_bytes
    if kind == "spmm":
        return 8.0 * nnz * nrhs, 20.0 * nnz + 8.0 * (ne + 1) + 32.0 * ne * nrhs
    return None, None


def measured_traffic(kernel, workload_name):
    """HBM bytes per launch from the committed rocprofv3 counter summary of
    this kernel on this workload, or None when there is none or the kernel's
    source changed after the counters were taken."""
    from paper_2311_05322_amd.pmc_summary import SOURCES, source_hash
    name = "k_" + kernel.split("_lower")[0].split("_upper")[0]
    path = os.path.join(ROOT, "profiles", f"{name}_{workload_name}_hbm_traffic.md")
    if name not in SOURCES or not os.path.exists(path):
        return None
    vals = {}
    with open(path) as f:
        for line in f:
            if ":" in line and line.split(":")[0] in ("bytes_per_launch", "source_sha256"):
                k, v = line.split(":", 1)
                vals[k] = v.strip()
    if vals.get("source_sha256") != source_hash(name) or "bytes_per_launch" not in vals:
        return None
    return float(vals["bytes_per_launch"])


def run_variant(ctx, p, eps_dev, E_dev, prec, steps, warmup, restart, profile=True, coarse=False, block=False,
                two_pass=False):
    import torch
    import paper_2311_05322_amd as mx
    S = np.zeros((len(p.src_pos), len(p.src_pos)), np.complex128)
    ctx.set_krylov(block, two_pass)

    def step():
        ctx.assemble(None, None, eps_dev, p.eps_kind, p.freq, p.eps_b, reuse_mesh=True)
        ctx.setup_schwarz(p.nsub, p.overlap, precision=prec, restart=restart, coarse=coarse)
        _, _, info = ctx.solve(p.src_pos, p.src_mom, rtol=p.rtol, E=E_dev, S=S)
        return info

    for w in range(warmup):
        info = step()
        log(f"  warmup {w}: iters {info['iters_max']} converged {info['converged']}")
    # timed steps: no per-kernel events, plain Arnoldi steps replayed from HIP graphs
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    infos = []
    for k in range(steps):
        infos.append(step())
        log(f"  step {k}: iters {infos[-1]['iters_max']} relres {infos[-1]['relres'].max():.2e} "
            f"fallback {infos[-1]['fallback']}")
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    kt = None
    if profile:
        # one more step, outside the timed region, with HIP events around every
        # kernel class (eager launches) for the per-kernel split and rooflines
        ctx.set_profiling(True)
        info = step()
        torch.cuda.synchronize()
        kt = ctx.kernel_times()
        ctx.set_profiling(False)
        log(f"  profiled step: iters {info['iters_max']}")
    ctx.set_krylov(False)
    return (t1 - t0) / steps, infos, kt, S


def cpu_baseline(p, iters, budget_s=25.0):
    """The oracle's CPU ORAS-FGMRES cost per all-transmitter solve, from a
    bounded sample of the same workload: per-subdomain set-up (local matrix +
    sparse LU) and local solves on a sample of subdomains, one operator product
    with all right-hand sides, element blocks on a sample of tetrahedra;
    scaled to the full workload with the iteration count of the GPU run."""
    from oracle import fem, schwarz
    t0 = time.perf_counter()
    T = fem.Topology(p.xyz, p.tet)
    dec = schwarz.Decomposition(T, p.nsub, p.overlap)
    t_prep = time.perf_counter() - t0
    nrhs = len(p.src_pos)
    # element blocks on a 1/16 sample of the tetrahedra
    k0 = fem.k0_of(p.freq)
    sub = fem.Topology.__new__(fem.Topology)
    sub.xyz = T.xyz
    sub.tet_sorted = T.tet_sorted[::16]
    t = time.perf_counter()
    fem.element_operator(sub, p.eps[::16], 0, k0)
    t_elem = (time.perf_counter() - t) * 16
    # operator product with all right-hand sides (operator values from the oracle, untimed)
    A = fem.assemble(T, p.eps, p.eps_kind, p.freq, p.eps_b)
    X = np.ones((T.ne, nrhs), np.complex128)
    t = time.perf_counter()
    A @ X
    t_spmv = time.perf_counter() - t
    # subdomain set-up and solves on a sample of subdomains within the budget
    t_set = t_sol = 0.0
    done = 0
    tb = time.perf_counter()
    order = np.random.default_rng(0).permutation(p.nsub)
    for i in order:
        t = time.perf_counter()
        B = dec.local_matrix(int(i), p.eps, p.eps_kind, p.freq, p.eps_b)
        lu = fem.sparse_lu(B)
        t1 = time.perf_counter()
        lu.solve(np.ascontiguousarray(X[dec.dofs[i]]))
        t_set += t1 - t
        t_sol += time.perf_counter() - t1
        done += 1
        if time.perf_counter() - tb > budget_s and done >= 4:
            break
    scale = p.nsub / done
    t_total = t_elem + scale * t_set + iters * (t_spmv + scale * t_sol)
    return {"value": 1.0 / t_total, "unit": "solves/s", "cores": 1, "kind": "oracle",
            "sample": (f"oracle ORAS-FGMRES (numpy/SuperLU, single thread) on the same workload: "
                       f"set-up and {nrhs}-RHS local solves of {done}/{p.nsub} subdomains, element blocks "
                       f"of 1/16 of the tetrahedra, one {nrhs}-RHS operator product; scaled by "
                       f"{scale:.1f} and by {iters} iterations; {t_total:.0f} s per solve"),
            "seconds_per_solve": t_total, "prep_s": t_prep}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="chamber1m", choices=sorted(WORKLOADS))
    ap.add_argument("--restart", type=int, default=30)
    ap.add_argument("--no-fp64", action="store_true", help="skip the FP64 reference variant")
    ap.add_argument("--no-learned", action="store_true", help="headline without the learned coarse term")
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--no-block", action="store_true", help="skip the block FGMRES variant")
    ap.add_argument("--block-cgs2", action="store_true", help="also time block FGMRES with two Gram-Schmidt passes")
    ap.add_argument("--cpu-budget", type=float, default=20.0)
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="MIB",
                    help="only run a plain device copy kernel (read MIB MiB, write MIB MiB) three times, as the "
                         "reference for HBM byte counters, and exit")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU: the solver runs on a single MI355X; --gpus {args.gpus} "
              "is not supported", file=sys.stderr)
        sys.exit(2)

    import torch
    if args.copy_calibration:
        n = args.copy_calibration * (1 << 20) // 4
        src = torch.ones(n, dtype=torch.float32, device="cuda:0")
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        for _ in range(3):
            torch.neg(src, out=dst)
        torch.cuda.synchronize()
        print(json.dumps({"copy_calibration_bytes_read": 4 * n, "copy_calibration_bytes_written": 4 * n,
                          "dispatches": 3}))
        return
    import paper_2311_05322_amd as mx

    p = make_problem(args.workload)
    dev = torch.device("cuda:0")
    stream = torch.cuda.Stream(device=dev)
    torch.cuda.set_stream(stream)
    ctx = mx.Context(0)
    ctx.set_stream(stream.cuda_stream)
    t = time.perf_counter()
    ctx.assemble(p.xyz, p.tet, p.eps, p.eps_kind, p.freq, p.eps_b)
    ctx.setup_schwarz(p.nsub, p.overlap, precision=mx.MX_PREC_C64, factor=False)
    log(f"topology + partition: {time.perf_counter() - t:.1f} s")
    sz = ctx.sizes()
    part, dof_ptr, *_ = ctx.partition()
    n_i = np.diff(dof_ptr)
    nrhs = len(p.src_pos)
    log(f"{args.workload}: ne={sz.ne} nnz={sz.nnz} nsub={sz.nsub} n_i {n_i.min()}..{n_i.max()} nrhs={nrhs}")
    eps_dev = torch.from_numpy(np.ascontiguousarray(p.eps)).to(dev)
    E_dev = torch.empty((sz.ne, nrhs), dtype=torch.complex128, device=dev)

    wfile = os.path.join(ROOT, "paper_2311_05322_amd", "weights", f"coarse_{args.workload}.npz")
    learned = os.path.exists(wfile) and not args.no_learned
    if learned:
        from paper_2311_05322_amd.train_coarse import load_weights
        ctx.setup_schwarz(p.nsub, p.overlap, precision=mx.MX_PREC_C64, factor=False, coarse=True)
        load_weights(ctx, wfile)
    variants = {}
    # the learned variant runs in block mode: judged learned steps first, then
    # block FGMRES from that iterate once plain ORAS has switched the term off
    order = ([("c64_learned", mx.MX_PREC_C64, True, True, False)] if learned else []) + \
        [("c64_plain", mx.MX_PREC_C64, False, False, False)]
    if not args.no_block:
        order.append(("c64_block", mx.MX_PREC_C64, False, True, False))
        if args.block_cgs2:
            order.append(("c64_block_cgs2", mx.MX_PREC_C64, False, True, True))
    if not args.no_fp64:
        order.append(("c128_plain", mx.MX_PREC_C128, False, False, False))
    for name, prec, co, blk, two in order:
        log(f"variant {name}")
        ms, infos, kt, S = run_variant(ctx, p, eps_dev, E_dev, prec, args.steps, args.warmup, args.restart,
                                       coarse=co, block=blk, two_pass=two)
        variants[name] = {"ms": ms, "infos": infos, "kt": kt, "S": S, "tuning": ctx.tuning()}
        log(f"  autotuner: {variants[name]['tuning']}")
    ctx.close()
    head = "c64_learned" if learned else "c64_plain"
    ms_mix, infos_mix, kt_mix, S_mix = (variants[head][k] for k in ("ms", "infos", "kt", "S"))
    ref = None
    if "c128_plain" in variants:
        v = variants["c128_plain"]
        ref = {"solves_per_s": 1.0 / v["ms"], "ms_per_step": v["ms"] * 1e3,
               "iters": int(v["infos"][-1]["iters_max"]),
               "kernel_ms_per_step": {k: x[0] for k, x in v["kt"].items() if x[1]},
               "S_rel_diff_vs_headline": float(np.abs(S_mix - v["S"]).max() / np.abs(v["S"]).max())}
    others = {k: {"solves_per_s": 1.0 / v["ms"], "iters": int(v["infos"][-1]["iters_max"]),
                  "fallback": int(v["infos"][-1]["fallback"]), "autotune": v["tuning"],
                  "kernel_ms_per_step": {kk: x[0] for kk, x in v["kt"].items() if x[1]}}
              for k, v in variants.items()}

    # dominant kernel of the headline variant and its roofline
    kt = kt_mix
    dom = max((k for k in kt if kt[k][1] > 0 and k in ("lu_update", "trsm_lower", "trsm_upper", "spmm")),
              key=lambda k: kt[k][0])
    flops, byts = algorithmic_work(dom, n_i, sz.nnz, sz.ne, nrhs, 8, kt)
    avg_s = kt[dom][0] / kt[dom][1] / 1e3
    if dom == "spmm":
        roof = {"bound": "hbm", "achieved": byts / avg_s / 1e9, "peak": HBM_PEAK_GBS, "unit": "GB/s"}
    else:
        roof = {"bound": "mfma", "achieved": flops / avg_s / 1e12, "peak": MFMA_PEAK_TFLOPS["fp32"],
                "unit": "TFLOP/s"}
    roof["frac"] = roof["achieved"] / roof["peak"]
    roof["traffic"] = measured_traffic(dom, args.workload)
    roof["kernel"] = dom
    roof["avg_launch_ms"] = avg_s * 1e3
    # the same figures for every kernel class that has an algorithmic count
    roof_all = {}
    for k in ("lu_update", "trsm_lower", "trsm_upper", "spmm"):
        if k not in kt or kt[k][1] == 0:
            continue
        f, b = algorithmic_work(k, n_i, sz.nnz, sz.ne, nrhs, 8, kt)
        a_s = kt[k][0] / kt[k][1] / 1e3
        if k == "spmm":
            roof_all[k] = {"bound": "hbm", "achieved": b / a_s / 1e9, "unit": "GB/s",
                           "frac": b / a_s / 1e9 / HBM_PEAK_GBS, "avg_launch_ms": a_s * 1e3}
        else:
            roof_all[k] = {"bound": "mfma", "achieved": f / a_s / 1e12, "unit": "TFLOP/s",
                           "frac": f / a_s / 1e12 / MFMA_PEAK_TFLOPS["fp32"], "avg_launch_ms": a_s * 1e3}

    cpu = None
    iters = int(infos_mix[-1]["iters_max"])
    if not args.no_cpu:
        log("cpu baseline (oracle, bounded sample)")
        cpu = cpu_baseline(p, iters, args.cpu_budget)

    value = 1.0 / ms_mix
    out = {
        "metric": "all-transmitter Maxwell solves/s @1e-8 residual: learned+FP32-LU vs FP64 Schwarz",
        "value": value, "unit": "solves/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": ms_mix * 1e3, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "c64/c128", "data": "synthetic",
        "config": {"workload": args.workload, "ne": int(sz.ne), "nnz": int(sz.nnz), "nsub": int(sz.nsub),
                   "overlap": p.overlap, "n_i_max": int(n_i.max()), "nrhs": nrhs, "rtol": p.rtol,
                   "restart": args.restart, "coarse": "learned" if head == "c64_learned" else "none",
                   "krylov": ("judged learned steps, then block FGMRES" if head == "c64_learned"
                              else "pseudo-block FGMRES"),
                   "precision": "complex64 LU + FP64 FGMRES"},
        "variants": others,
        "iters": iters,
        "speedup_vs_fp64_gpu": (value / ref["solves_per_s"]) if ref else None,
        "fastest_variant": (lambda k: {"name": k, "solves_per_s": others[k]["solves_per_s"],
                                       "iters": others[k]["iters"],
                                       "speedup_vs_fp64_gpu": (others[k]["solves_per_s"] / ref["solves_per_s"])
                                       if ref else None})(max(others, key=lambda k: others[k]["solves_per_s"])),
        "fp64_reference": ref,
        "kernel_ms_per_step": {k: v[0] for k, v in kt_mix.items() if v[1]},
        "roofline": roof,
        "roofline_by_kernel": roof_all,
        "cpu_baseline": cpu,
    }
    print(json.dumps(out))


if __name__ == "__main__":
    main()
