"""Pins of the learned-term oracle against an independent construction of the
same network in PyTorch (CPU, float64): GELU in its tanh form and its
derivative, the forward pass (plain and with bf16 rounding of every product
operand), the mean-squared-error loss and its parameter gradient by autograd,
and the Adam update against torch.optim.Adam.

The torch side is written from the network's definition (Linear layers,
torch's own GELU, neighbour mean as a row-normalised adjacency matrix,
torch's float32 -> bfloat16 conversion), shares no code with the oracle, and
so catches a wrong constant, a transposed weight, a wrong neighbour set or a
misplaced rounding in the oracle."""
import numpy as np
import pytest

import workload
from oracle import fem, learned, schwarz

torch = pytest.importorskip("torch")
F = torch.nn.functional


@pytest.fixture(scope="module")
def graph():
    p = workload.cube_problem(n=6, nsub=8, overlap=1)
    t = fem.Topology(p.xyz, p.tet)
    dec = schwarz.Decomposition(t, 8, 1)
    nb = [dec.neighbours(i) for i in range(dec.nsub)]
    # row-normalised adjacency built from the dof sets directly (shares a dof, not itself)
    n = dec.nsub
    A = np.zeros((n, n))
    sets = [set(dec.dofs[i].tolist()) for i in range(n)]
    for i in range(n):
        for j in range(n):
            if i != j and sets[i] & sets[j]:
                A[i, j] = 1.0
    A /= np.maximum(A.sum(1, keepdims=True), 1.0)
    return nb, torch.tensor(A, dtype=torch.float64)


def torch_params(theta):
    """Split the flat vector in the documented order W1 b1 ... Ws2 Wn2 b6."""
    th = torch.tensor(np.asarray(theta, np.float64), dtype=torch.float64)
    out, o = {}, 0
    for name, shp in [("W1", (256, 384)), ("b1", (256,)), ("W2", (256, 256)), ("b2", (256,)),
                      ("W3", (256, 256)), ("b3", (256,)), ("W4", (256, 256)), ("b4", (256,)),
                      ("Ws1", (256, 256)), ("Wn1", (256, 256)), ("b5", (256,)),
                      ("Ws2", (384, 256)), ("Wn2", (384, 256)), ("b6", (384,))]:
        k = int(np.prod(shp))
        out[name] = th[o:o + k].reshape(shp).clone().requires_grad_(True)
        o += k
    assert o == th.numel()
    return out


def torch_net(P, X, Anorm, rounding):
    r = (lambda a: a.float().bfloat16().double()) if rounding else (lambda a: a)
    act = lambda z: F.gelu(z, approximate="tanh")
    h = X
    for l in (1, 2, 3, 4):
        h = act(F.linear(r(h), r(P[f"W{l}"]), P[f"b{l}"]))
    m = torch.einsum("ij,gjf->gif", Anorm, h)
    h5 = act(F.linear(r(h), r(P["Ws1"])) + F.linear(r(m), r(P["Wn1"]), P["b5"]))
    m5 = torch.einsum("ij,gjf->gif", Anorm, h5)
    return F.linear(r(h5), r(P["Ws2"])) + F.linear(r(m5), r(P["Wn2"]), P["b6"])


def test_gelu_matches_torch():
    z = np.linspace(-8, 8, 2001)
    zt = torch.tensor(z, dtype=torch.float64, requires_grad=True)
    y = F.gelu(zt, approximate="tanh")
    (g,) = torch.autograd.grad(y.sum(), zt)
    assert np.abs(learned.gelu(z) - y.detach().numpy()).max() <= 1e-15 * 8
    assert np.abs(learned.gelu_grad(z) - g.numpy()).max() <= 1e-14


@pytest.mark.parametrize("rounding", [False, True])
def test_forward_matches_torch(graph, rounding):
    nb, Anorm = graph
    rng = np.random.default_rng(11)
    theta = learned.init_params(5, out_scale=1.0)
    X = rng.standard_normal((2, len(nb), learned.NIN))
    out, _ = learned.forward(theta, X, nb, use_bf16=rounding)
    ref = torch_net(torch_params(theta), torch.tensor(X), Anorm, rounding).detach().numpy()
    # identical arithmetic up to summation order (FP64 accumulations)
    assert np.abs(out - ref).max() <= 1e-12 * np.abs(ref).max()


def test_loss_gradient_matches_autograd(graph):
    nb, Anorm = graph
    rng = np.random.default_rng(12)
    theta = learned.init_params(6, out_scale=1.0)
    X = rng.standard_normal((3, len(nb), learned.NIN))
    Y = rng.standard_normal((3, len(nb), learned.NIN))
    L, g = learned.loss_and_grad(theta, X, Y, nb, use_bf16=False)
    P = torch_params(theta)
    out = torch_net(P, torch.tensor(X), Anorm, False)
    Lt = F.mse_loss(out, torch.tensor(Y))
    grads = torch.autograd.grad(Lt, list(P.values()))
    gt = np.concatenate([gg.numpy().ravel() for gg in grads])
    assert abs(L - Lt.item()) <= 1e-13 * abs(Lt.item())
    assert np.linalg.norm(g - gt) <= 1e-12 * np.linalg.norm(gt)
    # each parameter block separately (a swapped block would keep the norm)
    o = 0
    for name, gg in zip(P.keys(), grads):
        k = gg.numel()
        assert np.abs(g[o:o + k] - gg.numpy().ravel()).max() <= 1e-12 * (np.abs(gt).max()), name
        o += k


def test_adam_matches_torch():
    rng = np.random.default_rng(13)
    theta = rng.standard_normal(1000)
    m = np.zeros_like(theta)
    v = np.zeros_like(theta)
    w = torch.tensor(theta.copy(), dtype=torch.float64, requires_grad=True)
    opt = torch.optim.Adam([w], lr=2e-3, betas=(0.9, 0.999), eps=1e-8)
    for t in range(1, 6):
        g = rng.standard_normal(1000) * (10.0 ** -t)
        theta, m, v = learned.adam_step(theta, g, m, v, t, lr=2e-3)
        opt.zero_grad()
        w.grad = torch.tensor(g)
        opt.step()
        assert np.abs(theta - w.detach().numpy()).max() <= 1e-14 * np.abs(theta).max(), t
