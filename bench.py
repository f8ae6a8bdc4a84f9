#!/usr/bin/env python3
"""All-transmitter Maxwell solves per second on one MI355X.

One step = one all-transmitter solve for one permittivity map: operator
values (topology cached), dense ORAS subdomain matrices + batched LU, and
FGMRES of every transmitter to relative residual 1e-8 (true residual
checked; a step that does not reach it fails the run).  The headline variant
uses complex64 subdomain factors on the matrix cores under an FP64 outer
iteration; the plain FP64 one-level Schwarz solver is timed in the same run
as the reference, in both Krylov modes (pseudo-block: one FGMRES per
transmitter; block: one Krylov space for all transmitters), so the gain of
the precision and of the Krylov mode can be told apart. solves/s = 1 / median
step time; every variant's fields are compared with the FP64 solve.

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


def algorithmic_work(kind, sz, nrhs, elem_bytes, kt):
    """Algorithmic flops and bytes of one launch of a kernel class. The
    subdomain unknowns are in reverse Cuthill-McKee order and the
    factorisation and solves visit only the 64x64 tiles inside the band of
    each matrix; their work is what those tiles hold (tile counts from the
    library: sz.lu_tiles 64x64x64 complex tile products per factorisation,
    sz.trsm_tiles_lower / _upper 64x64 factor tiles per solve)."""
    if kind == "lu_update":
        tot = 8.0 * 64.0 ** 3 * sz.lu_tiles
        nfact = max(1, kt["lu_inv"][1] // 2)          # two timed intervals per factorisation
        return tot / max(1.0, kt["lu_update"][1] / nfact), None
    if kind in ("trsm_lower", "trsm_upper"):
        tiles = sz.trsm_tiles_lower if kind == "trsm_lower" else sz.trsm_tiles_upper
        return 8.0 * 64.0 * 64.0 * nrhs * tiles, 64.0 * 64.0 * elem_bytes * tiles
    if kind == "spmm":
        return 8.0 * sz.nnz * nrhs, 20.0 * sz.nnz + 8.0 * (sz.ne + 1) + 32.0 * sz.ne * nrhs
    return None, None


def measured_traffic(kernel, workload_name):
    """HBM bytes per launch from the committed rocprofv3 counter summary of
    this kernel on this workload, or None when there is none or the kernel's
    source changed after the counters were taken."""
    from paper_2311_05322_amd.pmc_summary import SOURCES, source_hash
    name = "k_" + kernel
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
    """Times `steps` all-transmitter solves (after `warmup` untimed ones), each
    bracketed by device synchronisation; returns the per-step wall times, the
    solve diagnostics, the per-kernel split of one more (profiled) step and S.
    Raises if a timed step does not reach the tolerance."""
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
    times, infos = [], []
    for k in range(steps):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        info = step()
        torch.cuda.synchronize()
        times.append(time.perf_counter() - t0)
        infos.append(info)
        log(f"  step {k}: {times[-1]:.3f} s iters {info['iters_max']} relres {info['relres'].max():.2e} "
            f"fallback {info['fallback']} (assemble {info['t_assemble']:.3f} s, set-up {info['t_setup']:.3f} s "
            f"of which LU {info['t_lu']:.3f} s, iterations {info['t_iter']:.3f} s)")
        if not info["converged"] or not np.all(info["relres"] <= p.rtol):
            raise RuntimeError(f"timed step {k} did not reach rtol {p.rtol}: converged {info['converged']}, "
                               f"max relres {info['relres'].max():.3e}")
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
    return times, infos, kt, S


_CPU = {}


def _cpu_worker_init():
    from threadpoolctl import threadpool_limits
    _CPU["limits"] = threadpool_limits(1)


def _cpu_subdomain(i):
    """Oracle set-up (local ORAS matrix + sparse LU) and one solve with all
    right-hand sides for subdomain i, in a worker process."""
    from oracle import fem
    p, dec, X = _CPU["p"], _CPU["dec"], _CPU["X"]
    t = time.perf_counter()
    B = dec.local_matrix(int(i), p.eps, p.eps_kind, p.freq, p.eps_b)
    lu = fem.sparse_lu(B)
    t1 = time.perf_counter()
    lu.solve(np.ascontiguousarray(X[dec.dofs[i]]))
    return t1 - t, time.perf_counter() - t1


def _cpu_rows(k):
    """The oracle's operator product on row block k of all right-hand sides."""
    Ak, X = _CPU["Ablocks"][k], _CPU["X"]
    t = time.perf_counter()
    Ak @ X
    return time.perf_counter() - t


def _cpu_elements(k):
    from oracle import fem
    T, p, ch = _CPU["T"], _CPU["p"], _CPU["tchunks"]
    sub = fem.Topology.__new__(fem.Topology)
    sub.xyz = T.xyz
    sub.tet_sorted = T.tet_sorted[ch[k]:ch[k + 1]]
    t = time.perf_counter()
    fem.element_operator(sub, p.eps[ch[k]:ch[k + 1]], 0, fem.k0_of(p.freq))
    return time.perf_counter() - t


def cpu_sample(p, budget_s=20.0, cores=None):
    """The oracle's CPU ORAS-FGMRES on a bounded sample of the same workload,
    in `cores` worker processes over subdomains (all host cores, at most 16):
    per-subdomain set-up (local matrix + sparse LU) and one all-transmitter
    local solve on a random sample of subdomains, the operator product with
    all right-hand sides and the element blocks split in row / tetrahedron
    chunks over the workers. Runs before the GPU is touched (the workers are
    forked)."""
    import multiprocessing as mp
    from oracle import fem, schwarz
    cores = cores or max(1, min(16, os.cpu_count() or 1))
    T = fem.Topology(p.xyz, p.tet)
    dec = schwarz.Decomposition(T, p.nsub, p.overlap)
    A = fem.assemble(T, p.eps, p.eps_kind, p.freq, p.eps_b).tocsr()
    nrhs = len(p.src_pos)
    X = np.ones((T.ne, nrhs), np.complex128)
    ch = np.linspace(0, T.ne, cores + 1).astype(np.int64)
    _CPU.update(p=p, dec=dec, X=X, T=T, Ablocks=[A[ch[k]:ch[k + 1]] for k in range(cores)],
                tchunks=np.linspace(0, T.nt, cores + 1).astype(np.int64))
    ctx = mp.get_context("fork")
    with ctx.Pool(cores, initializer=_cpu_worker_init) as pool:
        t = time.perf_counter()
        pool.map(_cpu_elements, range(cores))
        t_elem = time.perf_counter() - t
        t = time.perf_counter()
        pool.map(_cpu_rows, range(cores))
        t_spmm = time.perf_counter() - t
        order = np.random.default_rng(0).permutation(p.nsub)
        per = []
        t0 = time.perf_counter()
        for b in range(0, p.nsub, cores):
            per += pool.map(_cpu_subdomain, order[b:b + cores])
            if time.perf_counter() - t0 > budget_s:
                break
        t_sub = time.perf_counter() - t0
    done = len(per)
    set_sum = sum(x[0] for x in per)
    sol_sum = sum(x[1] for x in per)
    # wall time of the sampled batches, split between set-up and solves in
    # proportion to their summed per-subdomain times, scaled to all subdomains
    scale = p.nsub / done
    t_set = scale * t_sub * set_sum / (set_sum + sol_sum)
    t_sol = scale * t_sub * sol_sum / (set_sum + sol_sum)
    return {"cores": cores, "nrhs": nrhs, "done": done, "nsub": p.nsub, "t_elem": t_elem, "t_spmm": t_spmm,
            "t_set": t_set, "t_sol": t_sol}


def cpu_baseline(smp, iters):
    t_total = smp["t_elem"] + smp["t_set"] + iters * (smp["t_spmm"] + smp["t_sol"])
    return {"value": 1.0 / t_total, "unit": "solves/s", "cores": smp["cores"], "kind": "oracle",
            "sample": (f"oracle ORAS-FGMRES (numpy/SuperLU) in {smp['cores']} worker processes over subdomains "
                       f"on the same workload: local matrices, sparse LU and {smp['nrhs']}-RHS local solves of "
                       f"{smp['done']}/{smp['nsub']} subdomains (wall time scaled by {smp['nsub'] / smp['done']:.1f}), "
                       f"the element blocks and one {smp['nrhs']}-RHS operator product in {smp['cores']} chunks; "
                       f"{iters} iterations (those of the headline GPU run); {t_total:.0f} s per solve"),
            "seconds_per_solve": t_total}


def spmm_variants(p, reps, name, counts=(32, 16, 5)):
    """Every SpMM variant on the assembled operator: average launch time
    (the library's device events around each launch) at the given
    right-hand-side counts (at most 32), the rate against the algorithmic bytes, and the largest
    difference from variant 0."""
    import torch
    import paper_2311_05322_amd as mx
    ctx = mx.Context(0)
    ctx.assemble(p.xyz, p.tet, p.eps, p.eps_kind, p.freq, p.eps_b)
    sz = ctx.sizes()
    g = torch.Generator(device="cuda").manual_seed(0)
    X = torch.view_as_complex(torch.randn(ctx.ne, 32, 2, dtype=torch.float64, device="cuda", generator=g))
    out = {"workload": name, "ne": int(sz.ne), "nnz": int(sz.nnz), "reps": reps,
           "variants": {}}
    try:
        for nrhs in counts:
            Xn = X[:, :nrhs].contiguous()
            ref = None
            for v in (0, 1, 2):
                ctx.set_tuning(v, 1, 32)
                Y = ctx.apply_operator(Xn)
                ctx.set_profiling(True)
                for _ in range(reps):
                    ctx.apply_operator(Xn, Y)
                ms, n = ctx.kernel_times()["spmm"]
                ctx.set_profiling(False)
                ref = Y.clone() if ref is None else ref
                _, byts = algorithmic_work("spmm", sz, nrhs, 16, None)
                out["variants"][f"{nrhs}/{v}"] = {
                    "ms": ms / n, "GB_s": byts / (ms / n) / 1e6, "frac_hbm": byts / (ms / n) / 1e6 / HBM_PEAK_GBS,
                    "max_rel_diff_vs_0": float((Y - ref).abs().max() / ref.abs().max())}
                log(f"nrhs {nrhs} variant {v}: {ms / n:.4f} ms")
    finally:
        ctx.close()
    print(json.dumps(out))


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--ref-steps", type=int, default=5,
                    help="timed steps of the variants other than the headline (at most --steps)")
    ap.add_argument("--workload", default="chamber1m", choices=sorted(WORKLOADS))
    ap.add_argument("--restart", type=int, default=15)
    ap.add_argument("--no-fp64", action="store_true", help="skip the FP64 reference variants")
    ap.add_argument("--no-learned", action="store_true", help="headline without the learned coarse term")
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--no-block", action="store_true", help="skip the block FGMRES variants")
    ap.add_argument("--block-cgs2", action="store_true", help="also time block FGMRES with two Gram-Schmidt passes")
    ap.add_argument("--cpu-budget", type=float, default=20.0)
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="MIB",
                    help="only run a plain device copy kernel (read MIB MiB, write MIB MiB) three times, as the "
                         "reference for HBM byte counters, and exit")
    ap.add_argument("--spmm-variants", type=int, default=0, metavar="REPS",
                    help="only time every SpMM variant (REPS launches each, device events) at 32, 16 and 5 "
                         "right-hand sides on the workload's operator, print one JSON line and exit")
    ap.add_argument("--spmm-nrhs", default="32,16,5", help="right-hand-side counts of --spmm-variants")
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

    p = make_problem(args.workload)
    if args.spmm_variants:
        spmm_variants(p, args.spmm_variants, args.workload, [int(x) for x in args.spmm_nrhs.split(",")])
        return
    smp = None
    if not args.no_cpu:
        # the oracle's sample runs first, in forked workers, before the GPU is touched
        log("cpu baseline sample (oracle, all host cores)")
        t = time.perf_counter()
        smp = cpu_sample(p, args.cpu_budget)
        log(f"  {smp['done']} subdomains in {time.perf_counter() - t:.1f} s on {smp['cores']} cores")

    import paper_2311_05322_amd as mx
    dev = torch.device("cuda:0")
    stream = torch.cuda.Stream(device=dev)
    torch.cuda.set_stream(stream)
    ctx = mx.Context(0, stream=stream.cuda_stream)
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
    # (name, precision, learned term, block Krylov, two-pass)
    # the learned variant runs in block mode: judged learned steps first, then
    # block FGMRES from that iterate once plain ORAS has switched the term off
    order = ([("c64_learned", mx.MX_PREC_C64, True, True, False)] if learned else []) + \
        [("c64_plain", mx.MX_PREC_C64, False, False, False)]
    if not args.no_block:
        order.append(("c64_block", mx.MX_PREC_C64, False, True, False))
        if args.block_cgs2:
            order.append(("c64_block_cgs2", mx.MX_PREC_C64, False, True, True))
    if not args.no_fp64:
        if not args.no_block:
            order.append(("c128_block", mx.MX_PREC_C128, False, True, False))
        order.append(("c128_plain", mx.MX_PREC_C128, False, False, False))
    head = order[0][0]
    variants, fields = {}, {}
    for name, prec, co, blk, two in order:
        log(f"variant {name}")
        steps = args.steps if name == head else max(1, min(args.steps, args.ref_steps))
        warm = args.warmup if name == head else min(args.warmup, 1)
        times, infos, kt, S = run_variant(ctx, p, eps_dev, E_dev, prec, steps, warm, args.restart,
                                          coarse=co, block=blk, two_pass=two)
        variants[name] = {"times": times, "infos": infos, "kt": kt, "S": S, "tuning": ctx.tuning(),
                          "sizes": ctx.sizes()}
        fields[name] = E_dev.clone()
        log(f"  median {np.median(times):.3f} s, autotuner: {variants[name]['tuning']}")
    ctx.close()

    def field_err(name, ref):
        d = torch.linalg.vector_norm(fields[name] - fields[ref], dim=0)
        r = torch.linalg.vector_norm(fields[ref], dim=0)
        return float((d / r).max())

    fp64 = "c128_plain" if "c128_plain" in fields else None
    others = {}
    for k, v in variants.items():
        last = v["infos"][-1]
        others[k] = {"solves_per_s": 1.0 / float(np.median(v["times"])),
                     "s_per_solve_median": float(np.median(v["times"])),
                     "s_per_solve_mean": float(np.mean(v["times"])), "steps": len(v["times"]),
                     "iters": int(last["iters_max"]), "fallback": int(last["fallback"]),
                     "max_true_relres": float(max(i["relres"].max() for i in v["infos"])),
                     "phases_s": {"assemble": last["t_assemble"], "setup": last["t_setup"], "lu": last["t_lu"],
                                  "iterations": last["t_iter"]},
                     "field_rel_err_vs_fp64": field_err(k, fp64) if fp64 else None,
                     "autotune": v["tuning"],
                     "band_tiles": {"lu": int(v["sizes"].lu_tiles), "trsm_lower": int(v["sizes"].trsm_tiles_lower),
                                    "trsm_upper": int(v["sizes"].trsm_tiles_upper)},
                     "kernel_ms_per_step": {kk: x[0] for kk, x in v["kt"].items() if x[1]}}
    ms_mix = float(np.median(variants[head]["times"]))
    kt_mix = variants[head]["kt"]
    infos_mix = variants[head]["infos"]

    def ratio(a, b):
        return others[a]["solves_per_s"] / others[b]["solves_per_s"] if a in others and b in others else None

    ref = None
    if fp64:
        v = others[fp64]
        ref = {"solves_per_s": v["solves_per_s"], "ms_per_step": v["s_per_solve_median"] * 1e3,
               "iters": v["iters"], "kernel_ms_per_step": v["kernel_ms_per_step"],
               "S_rel_diff_vs_headline": float(np.abs(variants[head]["S"] - variants[fp64]["S"]).max()
                                               / np.abs(variants[fp64]["S"]).max())}

    # dominant kernel of the headline variant and its roofline
    kt = kt_mix
    dom = max((k for k in kt if kt[k][1] > 0 and k in ("lu_update", "trsm_lower", "trsm_upper", "spmm")),
              key=lambda k: kt[k][0])
    flops, byts = algorithmic_work(dom, variants[head]["sizes"], nrhs, 8, kt)
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
        f, b = algorithmic_work(k, variants[head]["sizes"], nrhs, 8, kt)
        a_s = kt[k][0] / kt[k][1] / 1e3
        if k == "spmm":
            roof_all[k] = {"bound": "hbm", "achieved": b / a_s / 1e9, "unit": "GB/s",
                           "frac": b / a_s / 1e9 / HBM_PEAK_GBS, "avg_launch_ms": a_s * 1e3}
        else:
            roof_all[k] = {"bound": "mfma", "achieved": f / a_s / 1e12, "unit": "TFLOP/s",
                           "frac": f / a_s / 1e12 / MFMA_PEAK_TFLOPS["fp32"], "avg_launch_ms": a_s * 1e3}

    iters = int(infos_mix[-1]["iters_max"])
    cpu = cpu_baseline(smp, iters) if smp else None

    value = 1.0 / ms_mix
    learned_note = None
    if head == "c64_learned" and "c64_block" in others:
        learned_note = {"iters_with": others["c64_learned"]["iters"], "iters_block_without": others["c64_block"]["iters"],
                        "fallback_code": others["c64_learned"]["fallback"],
                        "solves_per_s_ratio_vs_block": ratio("c64_learned", "c64_block")}
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
                   "precision": "complex64 LU + FP64 FGMRES", "timing": "median of the timed steps"},
        "variants": others,
        "iters": iters,
        "field_rel_err_vs_fp64": others[head]["field_rel_err_vs_fp64"],
        "speedup_vs_fp64_gpu": ratio(head, fp64) if fp64 else None,
        "speedup_matched_krylov": {"c64_block_vs_c128_block": ratio("c64_block", "c128_block"),
                                   "c64_plain_vs_c128_plain": ratio("c64_plain", "c128_plain"),
                                   "headline_vs_c128_block": ratio(head, "c128_block")},
        "learned_term": learned_note,
        "fastest_variant": (lambda k: {"name": k, "solves_per_s": others[k]["solves_per_s"],
                                       "iters": others[k]["iters"],
                                       "speedup_vs_fp64_gpu": ratio(k, fp64) if fp64 else None})(
            max(others, key=lambda k: others[k]["solves_per_s"])),
        "fp64_reference": ref,
        "kernel_ms_per_step": {k: v[0] for k, v in kt_mix.items() if v[1]},
        "roofline": roof,
        "roofline_by_kernel": roof_all,
        "cpu_baseline": cpu,
    }
    print(json.dumps(out))


if __name__ == "__main__":
    main()
