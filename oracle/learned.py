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
* BF16 arithmetic: the operands of every matrix product (weights and
  activations) rounded to bfloat16 (round to nearest even), products
  accumulated in higher precision; biases, GELU and the loss are not rounded.

Pinned by: exact reproduction of linear fields by P_i (partition of unity of
the trilinear hats), the backward pass against central finite differences,
and bf16 rounding against numpy's float32 -> bfloat16 bit arithmetic spelled
out independently in the tests.
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


def lattice_prolongation(topo, dofs, lo, hi):
    """P [n, 192] of the edges `dofs` on the 4x4x4 lattice of the box [lo, hi]."""
    xa = topo.xyz[topo.edges[dofs, 0]]
    xb = topo.xyz[topo.edges[dofs, 1]]
    t = xb - xa
    sq, wq = np.polynomial.legendre.leggauss(3)
    sq = 0.5 * (sq + 1.0)
    wq = 0.5 * wq
    P = np.zeros((len(dofs), NCOARSE))
    span = (hi - lo) / (NPA - 1)
    for s, w in zip(sq, wq):
        x = xa + s * t
        xi = (x - lo) / span                                   # [n, 3] in [0, 3]
        psi = np.maximum(0.0, 1.0 - np.abs(xi[:, :, None] - np.arange(NPA)[None, None, :]))  # [n,3,4]
        phi = (psi[:, 0, :, None, None] * psi[:, 1, None, :, None] * psi[:, 2, None, None, :])  # [n,a,b,c]
        phi = phi.transpose(0, 3, 2, 1).reshape(len(dofs), NNODE)   # node = a + 4b + 16c
        P += w * (phi[:, :, None] * t[:, None, :]).reshape(len(dofs), NCOARSE)
    return P


class Coarse:
    """Per-subdomain lattices, prolongations and least-squares operators."""

    def __init__(self, dec):
        self.dec = dec
        topo = dec.topo
        self.P, self.G = [], []
        for i in range(dec.nsub):
            lo, hi = subdomain_box(topo, dec.tets[i])
            P = lattice_prolongation(topo, dec.dofs[i], lo, hi)
            PDP = P.T @ (dec.D[i][:, None] * P)
            lam = 1e-6 * np.trace(PDP) / NCOARSE
            self.P.append(P)
            self.G.append(np.linalg.inv(PDP + lam * np.eye(NCOARSE)))
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
            ci = c[:, i, :NCOARSE] + 1j * c[:, i, NCOARSE:]            # [nrhs, 192]
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


def forward(theta, X, nbrs, use_bf16=True):
    """Network outputs [G, nsub, 384] for inputs X [G, nsub, 384], and a cache."""
    p = unflatten(theta)
    r = bf16 if use_bf16 else (lambda a: np.asarray(a, dtype=np.float64))
    cache = {"X": X}
    h = X
    for l in (1, 2, 3, 4):
        z = r(h) @ r(p[f"W{l}"]).T + p[f"b{l}"]
        cache[f"in{l}"], cache[f"z{l}"] = h, z
        h = gelu(z)
    cache["h4"] = h
    m4 = neighbour_mean(h, nbrs)
    z5 = r(h) @ r(p["Ws1"]).T + r(m4) @ r(p["Wn1"]).T + p["b5"]
    cache["m4"], cache["z5"] = m4, z5
    h5 = gelu(z5)
    m5 = neighbour_mean(h5, nbrs)
    out = r(h5) @ r(p["Ws2"]).T + r(m5) @ r(p["Wn2"]).T + p["b6"]
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
