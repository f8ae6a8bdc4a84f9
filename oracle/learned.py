"""Learned coarse-space correction of the one-level Schwarz preconditioner.

TEST INFRASTRUCTURE ONLY (see the package docstring).

Not a method of the paper: the paper's preconditioner is one-level ORAS
(Sec. IV-C).  This component is the solver's own addition; its definition
(fixed here and mirrored by the GPU kernels):

* Coarse lattice of subdomain i: the axis-aligned bounding box [lo, hi] of the
  vertices of its overlapping tetrahedra, 4 x 4 x 4 nodes (corners included),
  node (a, b, c) -> index a + 4 b + 16 c, a complex 3-vector per node:
  192 complex coefficients, 384 real channels [Re | Im].
* Prolongation P_i [n_i x 192] (real): P[l, 3 node + k] =
  int_0^1 phi_node(x_a + s t) ds * t_k, t = x_b - x_a, phi the trilinear hat
  of the node; 3-point Gauss-Legendre in s defines the integral.
* Input of transmitter j:  s_j = ||v_j|| / sqrt(ne),  x_i = P_i^T R_i v_j / s_j.
* Network (per subdomain node, per transmitter):
    h = GELU(W1 x + b1), then three times h = GELU(W h + b)      (256 wide)
    h = GELU(Ws1 h + Wn1 mean_{nbr} h + b5)                       (message pass 1)
    c = Ws2 h + Wn2 mean_{nbr} h + b6                             (message pass 2, 384)
  GELU in its tanh form; "nbr" = subdomains sharing a DOF with i.
* Correction q = s_j sum_i R_i^T D_i P_i c_i, added to the ORAS output.
* Training target: c*_i minimising ||D_i^{1/2} (R_i (e - M^{-1} r)/s - P_i c)||^2
  + lam ||c||^2, lam = 1e-6 tr(P^T D P)/192, for residual/error pairs (r, e)
  of the plain solver; loss = mean over nodes and channels of (c - c*)^2.
* Inside FGMRES the correction enters as z = M^{-1} v + theta_j q_j with one
  complex weight per transmitter minimising ||v_j - A z_j|| (theta_combination).
* BF16 arithmetic: the operands of every matrix product (weights and
  activations) rounded to bfloat16 (round to nearest even), products
  accumulated in higher precision; biases, GELU and the loss are not rounded.
* Optimiser: Adam on FP32 master weights.

Pinned by: exact reproduction of linear fields by P_i (partition of unity of
the trilinear hats); GELU, the forward pass (with and without bf16 rounding),
the loss and its parameter gradient against an independent PyTorch
construction of the same network (torch's GELU, autograd, torch's bfloat16
conversion); the backward pass against central finite differences; Adam
against torch.optim.Adam; bf16 rounding against bit arithmetic spelled out
in the tests; theta as the least-squares weight (orthogonality of the
residual it leaves, no perturbed weight does better).
"""
from __future__ import annotations

import numpy as np

NPA = 4                      # lattice nodes per axis
NNODE = NPA ** 3
NCOARSE = 3 * NNODE          # 192 complex coefficients
NIN = 2 * NCOARSE            # 384 real channels
WIDTH = 256

PARAM_SHAPES = [
    ("W1", (WIDTH, NIN)), ("b1", (WIDTH,)),
    ("W2", (WIDTH, WIDTH)), ("b2", (WIDTH,)),
    ("W3", (WIDTH, WIDTH)), ("b3", (WIDTH,)),
    ("W4", (WIDTH, WIDTH)), ("b4", (WIDTH,)),
    ("Ws1", (WIDTH, WIDTH)), ("Wn1", (WIDTH, WIDTH)), ("b5", (WIDTH,)),
    ("Ws2", (NIN, WIDTH)), ("Wn2", (NIN, WIDTH)), ("b6", (NIN,)),
]
NPARAM = sum(int(np.prod(s)) for _, s in PARAM_SHAPES)


def unflatten(theta):
    out, o = {}, 0
    for name, shp in PARAM_SHAPES:
        n = int(np.prod(shp))
        out[name] = np.asarray(theta[o:o + n], dtype=np.float64).reshape(shp)
        o += n
    return out


def flatten(p):
    return np.concatenate([np.asarray(p[name], dtype=np.float64).ravel() for name, _ in PARAM_SHAPES])


def init_params(seed=0, out_scale=0.1):
    """Normal(0, 1/fan_in) weights, zero biases, output layers scaled down."""
    rng = np.random.default_rng(seed)
    p = {}
    for name, shp in PARAM_SHAPES:
        if name.startswith("b"):
            p[name] = np.zeros(shp)
        else:
            p[name] = rng.standard_normal(shp) / np.sqrt(shp[1])
            if name in ("Ws2", "Wn2"):
                p[name] *= out_scale
    return flatten(p).astype(np.float32).astype(np.float64)


def bf16(x):
    """Round to bfloat16 (round to nearest, ties to even), returned as float64."""
    f = np.asarray(x, dtype=np.float32)
    u = f.view(np.uint32).astype(np.uint64)
    r = (u + 0x7FFF + ((u >> 16) & 1)) >> 16 << 16
    return (r.astype(np.uint32)).view(np.float32).astype(np.float64)


def gelu(z):
    a = np.sqrt(2.0 / np.pi)
    return 0.5 * z * (1.0 + np.tanh(a * (z + 0.044715 * z ** 3)))


def gelu_grad(z):
    a = np.sqrt(2.0 / np.pi)
    u = a * (z + 0.044715 * z ** 3)
    t = np.tanh(u)
    return 0.5 * (1.0 + t) + 0.5 * z * (1.0 - t * t) * a * (1.0 + 3 * 0.044715 * z * z)


# --------------------------------------------------------------------------
# coarse lattice
# --------------------------------------------------------------------------

def subdomain_box(topo, tets):
    v = np.unique(topo.tet_sorted[tets])
    X = topo.xyz[v]
    return X.min(axis=0), X.max(axis=0)


def lattice_prolongation(topo, dofs, lo, hi, npa=NPA):
    """P [n, 3 npa^3] of the edges `dofs` on the npa x npa x npa lattice of the
    box [lo, hi] (npa = 4: the network's 192 coefficients)."""
    xa = topo.xyz[topo.edges[dofs, 0]]
    xb = topo.xyz[topo.edges[dofs, 1]]
    t = xb - xa
    sq, wq = np.polynomial.legendre.leggauss(3)
    sq = 0.5 * (sq + 1.0)
    wq = 0.5 * wq
    nnode = npa ** 3
    P = np.zeros((len(dofs), 3 * nnode))
    span = (hi - lo) / (npa - 1)
    for s, w in zip(sq, wq):
        x = xa + s * t
        xi = (x - lo) / span                                   # [n, 3] in [0, npa - 1]
        psi = np.maximum(0.0, 1.0 - np.abs(xi[:, :, None] - np.arange(npa)[None, None, :]))  # [n,3,npa]
        phi = (psi[:, 0, :, None, None] * psi[:, 1, None, :, None] * psi[:, 2, None, None, :])  # [n,a,b,c]
        phi = phi.transpose(0, 3, 2, 1).reshape(len(dofs), nnode)   # node = a + npa b + npa^2 c
        P += w * (phi[:, :, None] * t[:, None, :]).reshape(len(dofs), 3 * nnode)
    return P


class Coarse:
    """Per-subdomain lattices, prolongations and least-squares operators
    (npa nodes per axis; the network uses npa = 4)."""

    def __init__(self, dec, npa=NPA):
        self.dec = dec
        self.ncoarse = 3 * npa ** 3
        topo = dec.topo
        self.P, self.G = [], []
        for i in range(dec.nsub):
            lo, hi = subdomain_box(topo, dec.tets[i])
            P = lattice_prolongation(topo, dec.dofs[i], lo, hi, npa)
            PDP = P.T @ (dec.D[i][:, None] * P)
            lam = 1e-6 * np.trace(PDP) / self.ncoarse
            self.P.append(P)
            self.G.append(np.linalg.inv(PDP + lam * np.eye(self.ncoarse)))
        nb = [dec.neighbours(i) for i in range(dec.nsub)]
        self.neighbours = nb

    def scale(self, v):
        return np.linalg.norm(v, axis=0) / np.sqrt(v.shape[0])

    def pool(self, v):
        """Features [nrhs, nsub, 384] of the block v [ne, nrhs]."""
        s = self.scale(v)
        s = np.where(s > 0, s, 1.0)
        feats = []
        for i in range(self.dec.nsub):
            f = self.P[i].T @ v[self.dec.dofs[i]] / s[None, :]        # [192, nrhs] complex
            feats.append(np.concatenate([f.real, f.imag], axis=0).T)  # [nrhs, 384]
        return np.stack(feats, axis=1)

    def targets(self, r, e, Minv_r):
        """c* [nrhs, nsub, 384] for residual/error pairs (columns of r, e)."""
        s = self.scale(r)
        s = np.where(s > 0, s, 1.0)
        t = (e - Minv_r) / s[None, :]
        out = []
        for i in range(self.dec.nsub):
            ti = t[self.dec.dofs[i]]
            rhs = self.P[i].T @ (self.dec.D[i][:, None] * ti)          # [192, nrhs] complex
            c = self.G[i] @ rhs
            out.append(np.concatenate([c.real, c.imag], axis=0).T)
        return np.stack(out, axis=1)

    def correction(self, c, v):
        """q = s sum_i R_i^T D_i P_i c_i for network outputs c [nrhs, nsub, 384]."""
        s = self.scale(v)
        q = np.zeros(v.shape, dtype=np.complex128)
        for i in range(self.dec.nsub):
            ci = c[:, i, :self.ncoarse] + 1j * c[:, i, self.ncoarse:]  # [nrhs, ncoarse]
            q[self.dec.dofs[i]] += self.dec.D[i][:, None] * (self.P[i] @ ci.T)
        return q * s[None, :]


# --------------------------------------------------------------------------
# network
# --------------------------------------------------------------------------

def neighbour_mean(h, nbrs):
    """h [G, nsub, F] -> mean over the neighbours of each subdomain."""
    out = np.zeros_like(h)
    for i, nb in enumerate(nbrs):
        if len(nb):
            out[:, i] = h[:, nb].mean(axis=1)
    return out


def neighbour_mean_T(g, nbrs):
    """Adjoint of neighbour_mean."""
    out = np.zeros_like(g)
    for i, nb in enumerate(nbrs):
        if len(nb):
            out[:, nb] += g[:, i:i + 1] / len(nb)
    return out


def dense(h, W, b, use_bf16=True):
    """Pre-activation of one MLP layer: W h + b over the last axis, the
    operands of the product rounded to bf16 when use_bf16."""
    r = bf16 if use_bf16 else (lambda a: np.asarray(a, dtype=np.float64))
    return r(h) @ r(W).T + b


def message_pass(h, nbrs, Ws, Wn, b, use_bf16=True):
    """Pre-activation of one message-passing layer: Ws h_i + Wn mean_{j in N(i)} h_j + b,
    and the neighbour mean it used."""
    r = bf16 if use_bf16 else (lambda a: np.asarray(a, dtype=np.float64))
    m = neighbour_mean(h, nbrs)
    return r(h) @ r(Ws).T + r(m) @ r(Wn).T + b, m


def forward(theta, X, nbrs, use_bf16=True):
    """Network outputs [G, nsub, 384] for inputs X [G, nsub, 384], and a cache."""
    p = unflatten(theta)
    cache = {"X": X}
    h = X
    for l in (1, 2, 3, 4):
        z = dense(h, p[f"W{l}"], p[f"b{l}"], use_bf16)
        cache[f"in{l}"], cache[f"z{l}"] = h, z
        h = gelu(z)
    cache["h4"] = h
    z5, m4 = message_pass(h, nbrs, p["Ws1"], p["Wn1"], p["b5"], use_bf16)
    cache["m4"], cache["z5"] = m4, z5
    h5 = gelu(z5)
    out, m5 = message_pass(h5, nbrs, p["Ws2"], p["Wn2"], p["b6"], use_bf16)
    cache["h5"], cache["m5"] = h5, m5
    return out, cache


def loss_and_grad(theta, X, Y, nbrs, use_bf16=True):
    """Mean squared error over all outputs and its gradient w.r.t. theta."""
    p = unflatten(theta)
    r = bf16 if use_bf16 else (lambda a: np.asarray(a, dtype=np.float64))
    out, c = forward(theta, X, nbrs, use_bf16)
    n = out.size
    diff = out - Y
    loss = float(np.sum(diff * diff) / n)
    dout = 2.0 * diff / n
    g = {}

    def wgrad(dz, a):
        return np.einsum("gno,gni->oi", r(dz), r(a))

    g["b6"] = dout.sum(axis=(0, 1))
    g["Ws2"] = wgrad(dout, c["h5"])
    g["Wn2"] = wgrad(dout, c["m5"])
    dh5 = r(dout) @ r(p["Ws2"]) + neighbour_mean_T(r(dout) @ r(p["Wn2"]), nbrs)
    dz5 = dh5 * gelu_grad(c["z5"])
    g["b5"] = dz5.sum(axis=(0, 1))
    g["Ws1"] = wgrad(dz5, c["h4"])
    g["Wn1"] = wgrad(dz5, c["m4"])
    dh = r(dz5) @ r(p["Ws1"]) + neighbour_mean_T(r(dz5) @ r(p["Wn1"]), nbrs)
    for l in (4, 3, 2, 1):
        dz = dh * gelu_grad(c[f"z{l}"])
        g[f"b{l}"] = dz.sum(axis=(0, 1))
        g[f"W{l}"] = wgrad(dz, c[f"in{l}"])
        dh = r(dz) @ r(p[f"W{l}"])
    return loss, flatten(g)


def adam_step(theta, grad, m, v, t, lr=1e-3, b1=0.9, b2=0.999, eps=1e-8):
    """One Adam update (t = 1, 2, ...) on FP32 master weights."""
    m = b1 * m + (1 - b1) * grad
    v = b2 * v + (1 - b2) * grad * grad
    mh = m / (1 - b1 ** t)
    vh = v / (1 - b2 ** t)
    return theta - lr * mh / (np.sqrt(vh) + eps), m, v


# --------------------------------------------------------------------------
# use inside FGMRES
# --------------------------------------------------------------------------

def theta_combination(A, v, z1, q):
    """Preconditioned block z = z1 + theta_j q_j with one complex weight per
    column j minimising ||v_j - A z_j||_2 (least squares in the one unknown
    theta_j: theta_j = (A q_j)^H (v_j - A z1_j) / ||A q_j||^2, 0 when A q_j = 0).
    z1 is the one-level ORAS output and q the learned correction; with the
    weight the learned term can only lower that local residual."""
    t = v - A @ z1
    aq = A @ q
    nrm2 = np.sum(np.abs(aq) ** 2, axis=0)
    dot = np.sum(aq.conj() * t, axis=0)
    theta = np.where(nrm2 > 0, dot / np.where(nrm2 > 0, nrm2, 1.0), 0.0)
    return z1 + theta[None, :] * q, theta
