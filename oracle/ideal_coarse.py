"""Bound on what the learned coarse term can gain (TEST INFRASTRUCTURE ONLY:
an analysis on the oracle, run by hand; nothing on the product path imports it).

At every FGMRES step the learned term's output is replaced by the exact
least-squares coarse correction, i.e. the targets of the training loss
computed from the true error A^{-1} v: the best output any network could give
in the lattice space. Iteration counts of plain ORAS and of this ideal
two-level preconditioner are printed for lattices of 2..8 nodes per axis.

python -m oracle.ideal_coarse --c 0.012 --nsub 64
"""
from __future__ import annotations

import argparse
import time

import numpy as np

import workload
from oracle import fem, krylov, learned, schwarz


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--c", type=float, default=0.012)
    ap.add_argument("--nsub", type=int, default=64)
    ap.add_argument("--lattices", default="2,4,6,8")
    ap.add_argument("--nrhs", type=int, default=2)
    a = ap.parse_args()
    p = workload.chamber_problem(c=a.c, nsub=a.nsub, overlap=1, nsrc=8, tear_seed=0)
    t = fem.Topology(p.xyz, p.tet)
    A = fem.assemble(t, p.eps, 0, p.freq, p.eps_b).tocsr()
    dec = schwarz.Decomposition(t, a.nsub, 1)
    M = schwarz.ORAS(dec, p.eps, 0, p.freq, p.eps_b)
    B = fem.dipole_rhs(t, p.src_pos, p.src_mom, p.freq)
    lu = fem.sparse_lu(A)

    def its(prec):
        return [krylov.fgmres(lambda v: A @ v, prec, B[:, j], 1e-8, 30, 600)[1] for j in range(a.nrhs)]

    print("edges", t.ne, "plain ORAS iterations", its(M.apply), flush=True)
    for npa in (int(x) for x in a.lattices.split(",")):
        learned.NPA, learned.NNODE = npa, npa ** 3
        learned.NCOARSE, learned.NIN = 3 * npa ** 3, 6 * npa ** 3
        co = learned.Coarse(dec)

        def ideal(v):
            v2 = v[:, None]
            e = lu.solve(v2.astype(np.complex128))
            return M.apply(v) + co.correction(co.targets(v2, e, M.apply(v2)), v2)[:, 0]

        t0 = time.time()
        print(f"lattice {npa}^3: ideal two-level iterations {its(ideal)} ({time.time() - t0:.0f} s)", flush=True)


if __name__ == "__main__":
    main()
