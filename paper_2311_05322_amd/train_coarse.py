"""Trains the learned coarse correction on the GPU and writes its weights.

Residual/error pairs come from the plain one-level solver itself (complex64
factors, no learned term) on training phantoms whose tear seeds differ from
the evaluation phantom; training runs entirely in the library's kernels
(mx_coarse_collect / mx_coarse_train).  The weights file holds the flat FP32
parameter vector and the input/output scales (numpy .npz, no pickles).

python -m paper_2311_05322_amd.train_coarse --workload chamber1m --out weights/coarse_chamber1m.npz
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
sys.path.insert(0, ROOT)

import workload  # noqa: E402
import paper_2311_05322_amd as mx  # noqa: E402

SHAPES = {
    "chamber1m": dict(c=0.004, mesh_seed=0, nsub=512, overlap=1, nsrc=32),
    "chamber130k": dict(c=0.008, mesh_seed=0, nsub=64, overlap=1, nsrc=32),
    "chamber2m": dict(c=0.00316, mesh_seed=0, nsub=2048, overlap=1, nsrc=32),
}


def load_weights(ctx, path):
    z = np.load(path, allow_pickle=False)
    ctx.coarse_set_weights(z["theta"], float(z["in_scale"]), float(z["out_scale"]))


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--workload", default="chamber1m", choices=sorted(SHAPES))
    ap.add_argument("--train-seeds", default="1000,1001,1002,1003")
    ap.add_argument("--eval-seed", type=int, default=0)
    ap.add_argument("--snap-every", type=int, default=4)
    ap.add_argument("--snapshots", type=int, default=16)
    ap.add_argument("--epochs", type=int, default=40)
    ap.add_argument("--batch", type=int, default=8)
    ap.add_argument("--epochs-per-call", type=int, default=2, help="epochs per library call (progress lines)")
    ap.add_argument("--lr", type=float, default=1e-3)
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--out", default=None, help="default: weights/coarse_<workload>.npz next to this file")
    a = ap.parse_args()
    if a.out is None:
        a.out = os.path.join(HERE, "weights", f"coarse_{a.workload}.npz")
    shp = SHAPES[a.workload]
    ctx = mx.Context(0)
    first = True
    t0 = time.time()
    for k, ts in enumerate(int(x) for x in a.train_seeds.split(",")):
        p = workload.chamber_problem(tear_seed=ts, **shp)
        ctx.assemble(p.xyz, p.tet, p.eps, p.eps_kind, p.freq, p.eps_b, reuse_mesh=not first)
        ctx.setup_schwarz(p.nsub, p.overlap, precision=mx.MX_PREC_C64, coarse=True)
        if first:
            ctx.coarse_init(a.seed)
            ctx.coarse_clear()
            first = False
        n = ctx.coarse_collect(p.src_pos, p.src_mom, snap_every=a.snap_every, max_snapshots=a.snapshots,
                               rtol_exact=1e-10)
        print(f"[collect] tear seed {ts}: {n} snapshots ({time.time() - t0:.1f} s)", flush=True)
    t1 = time.time()
    hist = []
    for e0 in range(0, a.epochs, a.epochs_per_call):
        ne = min(a.epochs_per_call, a.epochs - e0)
        hist.extend(ctx.coarse_train(ne, a.batch, a.lr, a.seed + e0))
        print(f"[train] epochs {e0 + ne}/{a.epochs}: loss {hist[-1]:.4f} ({time.time() - t1:.1f} s)", flush=True)
    hist = np.asarray(hist)
    print(f"[train] {a.epochs} epochs in {time.time() - t1:.1f} s, loss {hist[0]:.4f} -> {hist[-1]:.4f}", flush=True)
    theta, sx, sy = ctx.coarse_weights()
    os.makedirs(os.path.dirname(a.out), exist_ok=True)
    np.savez(a.out, theta=theta, in_scale=np.float64(sx), out_scale=np.float64(sy),
             loss=hist, meta=np.array(json.dumps({"workload": a.workload, "train_seeds": a.train_seeds,
                                                   "snap_every": a.snap_every, "snapshots": a.snapshots,
                                                   "epochs": a.epochs, "batch": a.batch, "lr": a.lr})))
    # held-out phantom: iterations with and without the learned term
    p = workload.chamber_problem(tear_seed=a.eval_seed, **shp)
    ctx.assemble(None, None, p.eps, p.eps_kind, p.freq, p.eps_b, reuse_mesh=True)
    res = {}
    for coarse in (False, True):
        ctx.setup_schwarz(p.nsub, p.overlap, precision=mx.MX_PREC_C64, coarse=coarse)
        t = time.time()
        _, _, info = ctx.solve(p.src_pos, p.src_mom, rtol=1e-8, want_E=False)
        res["learned" if coarse else "plain"] = {"iters": int(info["iters_max"]), "seconds": time.time() - t,
                                                 "fallback": int(info["fallback"])}
    print("[eval]", json.dumps(res), flush=True)
    ctx.close()


if __name__ == "__main__":
    main()
