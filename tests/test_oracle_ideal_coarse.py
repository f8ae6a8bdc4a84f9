"""What the learned coarse term can gain at best, measured with the oracle.

At every FGMRES step the network output is replaced by the exact
least-squares lattice coefficients of the error that one-level ORAS leaves
(the training targets computed from the true error A^{-1} v): no network can
output anything better in that coarse space. The iteration counts bound the
gain of the learned term and show how it grows with the lattice: the
network's 4x4x4 lattice, a 6x6x6 and an 8x8x8 lattice, against plain ORAS on
a small chamber (9.4k edges, 16 subdomains)."""
import numpy as np
import pytest

import workload
from oracle import fem, krylov, learned, schwarz


def _ideal_iterations(p, nsub, lattices, nrhs=2):
    t = fem.Topology(p.xyz, p.tet)
    A = fem.assemble(t, p.eps, 0, p.freq, p.eps_b).tocsr()
    dec = schwarz.Decomposition(t, nsub, 1)
    M = schwarz.ORAS(dec, p.eps, 0, p.freq, p.eps_b)
    B = fem.dipole_rhs(t, p.src_pos, p.src_mom, p.freq)
    lu = fem.sparse_lu(A)

    def its(prec):
        return max(krylov.fgmres(lambda v: A @ v, prec, B[:, j], 1e-8, 30, 600)[1] for j in range(nrhs))

    out = {"plain": its(M.apply)}
    for npa in lattices:
        co = learned.Coarse(dec, npa)

        def ideal(v, co=co):
            v2 = v[:, None]
            e = lu.solve(v2.astype(np.complex128))
            Mv = M.apply(v2)
            return Mv[:, 0] + co.correction(co.targets(v2, e, Mv), v2)[:, 0]

        out[npa] = its(ideal)
    return out


@pytest.mark.slow
def test_ideal_coarse_correction_bounds_the_gain():
    p = workload.chamber_problem(c=0.02, nsub=16, overlap=1, nsrc=8, tear_seed=0)
    it = _ideal_iterations(p, 16, (4, 6, 8))
    print(it)
    # the exact correction never hurts, and more lattice nodes capture more of the error
    assert it[4] <= it["plain"]
    assert it[8] <= it[6] <= it[4]
    assert it[8] < it["plain"]
