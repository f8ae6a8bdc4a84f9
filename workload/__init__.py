"""Seeded synthetic inputs for the Maxwell/Schwarz solver and its oracle.

This module produces *inputs only*: tetrahedral meshes, per-tetrahedron or
per-vertex relative permittivities, and point-dipole positions.  It contains
none of the solver's arithmetic (no basis functions, no element matrices, no
linear algebra), so both the CPU oracle and the GPU path may import it.

The paper (Sec. IV-A) builds conformal meshes of a CAD shoulder with MMG;
neither the CAD model nor the mesher is available, so a seeded, jittered
Kuhn lattice clipped to a cylinder stands in for the chamber mesh, and a
shoulder-like phantom (bone, muscle, tendon, tear ellipsoid) assigns the
Table I tissue classes.  Permittivities use the paper's material law
eps_r = eps' - j sigma / (omega eps0) with the exp(+j omega t) convention
(Sec. IV-B).
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np

EPS0 = 8.8541878128e-12
MU0 = 4.0e-7 * math.pi
C0 = 299792458.0

# (eps', sigma [S/m]) at 1 GHz of the tissue classes used by the phantoms.
MATERIALS = {
    "matching": (44.0, 0.6),
    "bone": (12.0, 0.2),
    "muscle": (55.0, 0.95),
    "tendon": (45.0, 0.8),
    "tear": (68.0, 1.5),
    "inclusion": (12.0, 0.2),
}


def eps_r(eps_prime: float, sigma: float, freq_hz: float) -> complex:
    """Complex relative permittivity eps' - j sigma/(omega eps0) (Sec. IV-B)."""
    return complex(eps_prime, -sigma / (2.0 * math.pi * freq_hz * EPS0))


# --------------------------------------------------------------------------
# meshes
# --------------------------------------------------------------------------

# The six Kuhn (Freudenthal) simplices of the unit cube: each is the path
# 0 -> e_p0 -> e_p0+e_p1 -> (1,1,1) for a permutation p of the axes.  All cubes
# use the same split, so faces match across cubes (a conforming mesh).
_PERMS = [(0, 1, 2), (0, 2, 1), (1, 0, 2), (1, 2, 0), (2, 0, 1), (2, 1, 0)]


def kuhn_box(n, lo, hi):
    """Structured Kuhn mesh of the box [lo, hi] with n = (nx, ny, nz) cubes.

    Returns xyz [V,3] float64 and tet [T,4] int32 (vertex order = Kuhn path;
    orientation not normalised).  Vertex (i,j,k) has id i + (nx+1)(j + (ny+1)k).
    """
    nx, ny, nz = (int(v) for v in n)
    lo = np.asarray(lo, dtype=np.float64)
    hi = np.asarray(hi, dtype=np.float64)
    gx = lo[0] + (hi[0] - lo[0]) * np.arange(nx + 1) / nx
    gy = lo[1] + (hi[1] - lo[1]) * np.arange(ny + 1) / ny
    gz = lo[2] + (hi[2] - lo[2]) * np.arange(nz + 1) / nz
    Z, Y, X = np.meshgrid(gz, gy, gx, indexing="ij")
    xyz = np.stack([X.ravel(), Y.ravel(), Z.ravel()], axis=1)

    def vid(i, j, k):
        return i + (nx + 1) * (j + (ny + 1) * k)

    k, j, i = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    i = i.ravel(); j = j.ravel(); k = k.ravel()
    tets = []
    for p in _PERMS:
        cur = np.zeros(3, dtype=np.int64)
        path = [cur.copy()]
        for ax in p:
            cur[ax] += 1
            path.append(cur.copy())
        verts = [vid(i + q[0], j + q[1], k + q[2]) for q in path]
        tets.append(np.stack(verts, axis=1))
    # interleave so that the six tets of one cube are consecutive
    tet = np.stack(tets, axis=1).reshape(-1, 4)
    return xyz, tet.astype(np.int32)


def kuhn_cube(n: int, side: float = 0.1):
    """[0, side]^3 cut into n^3 cubes of six Kuhn tetrahedra each."""
    return kuhn_box((n, n, n), (0.0, 0.0, 0.0), (side, side, side))


def jittered_cylinder(radius: float, height: float, c: float, seed: int,
                      jitter: float = 0.1):
    """Seeded unstructured-like mesh of the cylinder x^2+y^2 < radius^2, 0<z<height.

    A Kuhn lattice of the bounding box with cube size about c; every vertex is
    moved by a seeded uniform offset in [-jitter*c, jitter*c]^3 (small enough
    that no tetrahedron inverts); tetrahedra whose jittered centroid lies in
    the cylinder are kept (staircase boundary), unused vertices are dropped.

    Numbering, as a mesher's locality reordering would leave it: vertices in
    Morton (Z-curve) order of their lattice position, tetrahedra in Morton
    order of their lattice cube (the six of one cube consecutive, in Kuhn path
    order). Each tetrahedron keeps its vertices in Kuhn path order.
    """
    nxy = int(math.ceil(2.0 * radius / c))
    nz = int(math.ceil(height / c))
    xyz, tet = kuhn_box((nxy, nxy, nz), (-radius, -radius, 0.0), (radius, radius, height))
    rng = np.random.default_rng(seed)
    hx = 2.0 * radius / nxy
    hz = height / nz
    h = min(hx, hz)
    xyz = xyz + rng.uniform(-jitter * h, jitter * h, size=xyz.shape)
    cen = xyz[tet].mean(axis=1)
    keep = cen[:, 0] ** 2 + cen[:, 1] ** 2 < radius * radius
    cube = np.nonzero(keep)[0] // 6
    ci, cj, ck = cube % nxy, (cube // nxy) % nxy, cube // (nxy * nxy)
    tet = tet[keep][np.argsort(morton3(ci, cj, ck), kind="stable")]
    used = np.zeros(xyz.shape[0], dtype=bool)
    used[tet.ravel()] = True
    vid = np.nonzero(used)[0]
    vi, vj, vk = vid % (nxy + 1), (vid // (nxy + 1)) % (nxy + 1), vid // ((nxy + 1) * (nxy + 1))
    vid = vid[np.argsort(morton3(vi, vj, vk), kind="stable")]
    newid = np.full(xyz.shape[0], -1, dtype=np.int64)
    newid[vid] = np.arange(vid.size)
    return np.ascontiguousarray(xyz[vid]), newid[tet].astype(np.int32)


def morton3(i, j, k):
    """Z-curve code of non-negative lattice indices (< 2^20 each): bits of
    i, j, k interleaved, i in the lowest position."""
    code = np.zeros(np.shape(i), dtype=np.int64)
    i, j, k = (np.asarray(a, dtype=np.int64) for a in (i, j, k))
    for b in range(20):
        code |= ((i >> b) & 1) << (3 * b)
        code |= ((j >> b) & 1) << (3 * b + 1)
        code |= ((k >> b) & 1) << (3 * b + 2)
    return code


# --------------------------------------------------------------------------
# phantoms (material labels at tetrahedron centroids or at vertices)
# --------------------------------------------------------------------------

def _in_ellipsoid(p, centre, semi):
    d = (p - np.asarray(centre)) / np.asarray(semi)
    return (d * d).sum(axis=1) <= 1.0


@dataclasses.dataclass
class Phantom:
    """Shoulder-like phantom inside the cylindrical chamber (lengths in m)."""
    tear_centre: tuple | None
    tear_semi: tuple | None
    muscle_centre: tuple = (0.0, 0.0, 0.10)
    muscle_semi: tuple = (0.070, 0.060, 0.080)
    bone_axis_xy: tuple = (0.010, 0.0)
    bone_radius: float = 0.015
    bone_z: tuple = (0.04, 0.13)
    tendon_lo: tuple = (-0.030, -0.025, 0.130)
    tendon_hi: tuple = (0.040, 0.025, 0.140)

    def labels(self, p):
        """Tissue class per point, precedence matching<muscle<bone<tendon<tear."""
        lab = np.zeros(p.shape[0], dtype=np.int8)
        lab[_in_ellipsoid(p, self.muscle_centre, self.muscle_semi)] = 1
        bx, by = self.bone_axis_xy
        r2 = (p[:, 0] - bx) ** 2 + (p[:, 1] - by) ** 2
        bone = (r2 <= self.bone_radius ** 2) & (p[:, 2] >= self.bone_z[0]) & (p[:, 2] <= self.bone_z[1])
        lab[bone] = 2
        lo = np.asarray(self.tendon_lo); hi = np.asarray(self.tendon_hi)
        lab[np.all((p >= lo) & (p <= hi), axis=1)] = 3
        if self.tear_centre is not None:
            lab[_in_ellipsoid(p, self.tear_centre, self.tear_semi)] = 4
        return lab


LABEL_NAMES = ["matching", "muscle", "bone", "tendon", "tear"]


def shoulder_phantom(tear_seed: int | None) -> Phantom:
    """Phantom with a seeded tear: diameter d ~ U(5,15) mm, semi-axes
    d/2*(1.2, 1, 0.8), centre uniform in the tendon slab.  None = healthy."""
    if tear_seed is None:
        return Phantom(None, None)
    rng = np.random.default_rng(10_000 + int(tear_seed))
    d = rng.uniform(0.005, 0.015)
    ph = Phantom(None, None)
    lo = np.asarray(ph.tendon_lo); hi = np.asarray(ph.tendon_hi)
    centre = tuple(rng.uniform(lo, hi))
    semi = (0.5 * d * 1.2, 0.5 * d, 0.5 * d * 0.8)
    return Phantom(centre, semi)


def eps_of_labels(lab, freq_hz: float):
    table = np.array([eps_r(*MATERIALS[name], freq_hz) for name in LABEL_NAMES])
    return table[lab]


def tet_centroids(xyz, tet):
    return xyz[tet].mean(axis=1)


# --------------------------------------------------------------------------
# sources
# --------------------------------------------------------------------------

def dipole_ring(n: int, radius: float, centre_xy, z: float, phase: float = 0.0):
    """n unit z-directed dipoles at angles 2*pi*k/n + phase on a horizontal ring."""
    th = 2.0 * math.pi * np.arange(n) / n + phase
    pos = np.stack([centre_xy[0] + radius * np.cos(th),
                    centre_xy[1] + radius * np.sin(th),
                    np.full(n, z)], axis=1)
    mom = np.zeros((n, 3), dtype=np.complex128)
    mom[:, 2] = 1.0
    return pos, mom


# --------------------------------------------------------------------------
# named problems
# --------------------------------------------------------------------------

@dataclasses.dataclass
class Problem:
    name: str
    xyz: np.ndarray          # [V,3] float64
    tet: np.ndarray          # [T,4] int32
    eps: np.ndarray          # [T] (P0) or [V] (P1) complex128
    eps_kind: int            # 0 = per tetrahedron, 1 = per vertex
    eps_b: complex           # background permittivity used on the outer boundary
    freq: float
    src_pos: np.ndarray      # [nrhs,3]
    src_mom: np.ndarray      # [nrhs,3] complex
    nsub: int
    overlap: int
    rtol: float
    meta: dict


def cube_problem(n: int = 8, seed: int = 0, nsub: int = 8, overlap: int = 1,
                 freq: float = 1e9, nsrc: int = 8) -> Problem:
    """Unit-cube problem: [0,0.1]^3 Kuhn mesh, lossy background, one seeded
    ellipsoidal inclusion in the inner half, a ring of z-dipoles at z=0.05."""
    xyz, tet = kuhn_cube(n, 0.1)
    rng = np.random.default_rng(seed)
    semi = np.array([0.012, 0.008, 0.010])
    centre = rng.uniform(0.025 + semi, 0.075 - semi)
    cen = tet_centroids(xyz, tet)
    inside = _in_ellipsoid(cen, centre, semi)
    eb = eps_r(*MATERIALS["matching"], freq)
    eps = np.full(tet.shape[0], eb, dtype=np.complex128)
    eps[inside] = eps_r(*MATERIALS["inclusion"], freq)
    pos, mom = dipole_ring(nsrc, 0.04, (0.05, 0.05), 0.05)
    return Problem(f"cube{n}", xyz, tet, eps, 0, eb, freq, pos, mom, nsub, overlap, 1e-8,
                   {"inclusion_centre": centre.tolist(), "inclusion_semi": semi.tolist(),
                    "n": n, "seed": seed})


def chamber_problem(c: float = 0.004, mesh_seed: int = 0, tear_seed: int | None = 0,
                    nsub: int = 256, overlap: int = 2, nsrc: int = 32,
                    rings: int = 1, eps_kind: int = 0, freq: float = 1e9,
                    radius: float = 0.12, height: float = 0.2,
                    ring_radius: float = 0.11) -> Problem:
    """Cylindrical chamber (radius 0.12 m, height 0.2 m) with the shoulder-like
    phantom; c is the lattice cube size (4 mm gives about 1.0M edges)."""
    xyz, tet = jittered_cylinder(radius, height, c, mesh_seed)
    ph = shoulder_phantom(tear_seed)
    if eps_kind == 0:
        lab = ph.labels(tet_centroids(xyz, tet))
    else:
        lab = ph.labels(xyz)
    eps = eps_of_labels(lab, freq)
    eb = eps_r(*MATERIALS["matching"], freq)
    if rings == 1:
        pos, mom = dipole_ring(nsrc, ring_radius, (0.0, 0.0), 0.10)
    else:
        ps, ms = [], []
        zs = 0.10 + 0.02 * (np.arange(rings) - (rings - 1) / 2.0)
        for r, z in enumerate(zs):
            p, m = dipole_ring(nsrc, ring_radius, (0.0, 0.0), float(z),
                               phase=(math.pi / nsrc) * (r % 2))
            ps.append(p); ms.append(m)
        pos, mom = np.concatenate(ps), np.concatenate(ms)
    return Problem(f"chamber_c{c*1000:g}mm", xyz, tet, eps, eps_kind, eb, freq, pos, mom,
                   nsub, overlap, 1e-8,
                   {"c": c, "mesh_seed": mesh_seed, "tear_seed": tear_seed,
                    "tear_centre": ph.tear_centre, "tear_semi": ph.tear_semi})


def batched_specs(n: int = 8, seed: int = 0):
    """Seeded specifications of n phantoms solved as one batch: lattice cube
    size c ~ U(3.6, 4.77) mm (about 1.4M to 0.6M edges in the chamber), mesh
    jitter seed and tear seed k, and the number of subdomains that keeps the
    overlapping subdomains between about 2.5k and 5.5k unknowns (512 below
    1.0M edges, 1024 above; the edge count is about 1.02M (4 mm / c)^3).
    Returns a list of dicts (c, mesh_seed, tear_seed, nsub)."""
    rng = np.random.default_rng(seed)
    out = []
    for k in range(n):
        c = float(rng.uniform(0.0036, 0.00477))
        ne_est = 1.02e6 * (0.004 / c) ** 3
        out.append({"c": c, "mesh_seed": k, "tear_seed": k, "nsub": 512 if ne_est < 1.0e6 else 1024})
    return out


@dataclasses.dataclass
class PortSpec:
    """Rectangular waveguide aperture on the mesh boundary: centre, outward
    unit normal, broad-side unit vector u (width a), height b along
    normal x u, relative permittivity eps of the guide's filling."""
    centre: tuple
    normal: tuple
    u: tuple
    a: float
    b: float
    eps: complex


def box_chamber(side: float, height: float, h: float, ports_per_wall: int = 4, rings=(0.4, 0.6),
                port_cells=(5, 2), eps_port: complex = 59.0):
    """Box chamber [-side/2, side/2]^2 x [0, height] for the waveguide-port
    model: a Kuhn lattice of cube size about h (Morton-numbered like
    jittered_cylinder, not jittered, so that the walls stay planar), and
    4 * ports_per_wall * len(rings) apertures of port_cells lattice cells
    (broad side horizontal, height along z) on the four side walls, spread
    evenly along each wall at the heights rings * height, snapped to lattice
    lines (ValueError if two apertures would overlap). The paper's antennas are ceramic-filled (eps_r = 59) open-ended
    guides on rings around the imaging domain (Sec. III)."""
    nxy = int(math.ceil(side / h))
    nz = int(math.ceil(height / h))
    xyz, tet = kuhn_box((nxy, nxy, nz), (-side / 2, -side / 2, 0.0), (side / 2, side / 2, height))
    hx, hz = side / nxy, height / nz
    cube = np.arange(tet.shape[0]) // 6
    ci, cj, ck = cube % nxy, (cube // nxy) % nxy, cube // (nxy * nxy)
    tet = tet[np.argsort(morton3(ci, cj, ck), kind="stable")]
    nv = xyz.shape[0]
    vid = np.arange(nv)
    vi, vj, vk = vid % (nxy + 1), (vid // (nxy + 1)) % (nxy + 1), vid // ((nxy + 1) * (nxy + 1))
    order = np.argsort(morton3(vi, vj, vk), kind="stable")
    newid = np.empty(nv, dtype=np.int64)
    newid[order] = np.arange(nv)
    xyz = np.ascontiguousarray(xyz[order])
    tet = newid[tet].astype(np.int32)
    pa, pb = port_cells
    a, b = pa * hx, pb * hz
    ks = [int(round(zr * nz - pb / 2)) for zr in rings]
    iss = [int(round((q + 0.5) * nxy / ports_per_wall - pa / 2)) for q in range(ports_per_wall)]
    for lo_hi, n_, w_ in ((sorted(ks), nz, pb), (iss, nxy, pa)):
        if lo_hi[0] < 0 or lo_hi[-1] + w_ > n_ or any(y - x < w_ for x, y in zip(lo_hi, lo_hi[1:])):
            raise ValueError("apertures overlap or leave the wall at this lattice size")
    ports = []
    for k0 in ks:
        zc = (k0 + pb / 2) * hz
        for w, (nrm, u) in enumerate((((1, 0, 0), (0, 1, 0)), ((0, 1, 0), (-1, 0, 0)),
                                      ((-1, 0, 0), (0, -1, 0)), ((0, -1, 0), (1, 0, 0)))):
            for i0 in iss:
                s = -side / 2 + (i0 + pa / 2) * hx      # position along u
                c = [nrm[0] * side / 2 + u[0] * s, nrm[1] * side / 2 + u[1] * s, zc]
                ports.append(PortSpec(tuple(c), nrm, u, a, b, complex(eps_port)))
    return xyz, tet, ports


def seeded_complex(shape, seed: int, scale: float = 1.0):
    """Seeded standard complex normal array (test vectors)."""
    rng = np.random.default_rng(seed)
    return scale * (rng.standard_normal(shape) + 1j * rng.standard_normal(shape))
