"""The reconstruction loop (L-BFGS over the GPU cost and adjoint gradient)
on a small chamber: every accepted step lowers the cost of eq. (4)."""
import numpy as np
import pytest

mx = pytest.importorskip("paper_2311_05322_amd")
from paper_2311_05322_amd.reconstruct import run_reconstruction  # noqa: E402

pytestmark = pytest.mark.gpu


def test_reconstruction_lowers_cost():
    print("[case] reconstruction c=20mm nsub=16 nsrc=8 iters=3", flush=True)
    out = run_reconstruction(c=0.02, nsub=16, nsrc=8, iters=3, verbose=False)
    h = out["history"]
    print(out)
    assert len(h) >= 2 and np.all(np.isfinite(h))
    assert all(b < a for a, b in zip(h, h[1:]))
    assert h[-1] < 0.9 * h[0]
