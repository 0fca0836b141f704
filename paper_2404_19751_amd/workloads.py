"""Seeded synthetic inputs: procedural triangle meshes and particle placements.

This module only *generates inputs*. It holds none of the method's arithmetic
(no half-edge structure, no unfolding, no geodesic, force or walk code), so the
HIP path and the CPU oracle can both read what it produces without sharing any
of the computation under test.

Particle positions follow the paper's representation: a face index plus a
barycentric triple of doubles (Sec. 3, description of mesh-space models).
Random numbers come from SplitMix64 (Steele, Lea & Flood, OOPSLA 2014), taking
the top 53 bits of each output as a double in [0, 1).

Every mesh is oriented counter-clockwise seen from outside (outward normals),
closed surfaces are 2-manifolds, open ones (grid, cone fan, prism, L-shape,
height field) have a boundary.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

_MASK64 = (1 << 64) - 1
_GOLDEN_GAMMA = 0x9E3779B97F4A7C15


# --------------------------------------------------------------------------
# SplitMix64
# --------------------------------------------------------------------------
def splitmix64(seed: int, n: int) -> np.ndarray:
    """The first ``n`` outputs of SplitMix64 started from state ``seed``.

    The state advances by the golden gamma before each output; the output is
    the state passed through the two xor-shift-multiply mixing rounds.
    """
    k = np.arange(1, n + 1, dtype=np.uint64)
    with np.errstate(over="ignore"):
        z = np.uint64(seed & _MASK64) + k * np.uint64(_GOLDEN_GAMMA)
        z = (z ^ (z >> np.uint64(30))) * np.uint64(0xBF58476D1CE4E5B9)
        z = (z ^ (z >> np.uint64(27))) * np.uint64(0x94D049BB133111EB)
        z = z ^ (z >> np.uint64(31))
    return z


def uniforms(seed: int, n: int) -> np.ndarray:
    """``n`` doubles in [0, 1) from the top 53 bits of SplitMix64 outputs."""
    return (splitmix64(seed, n) >> np.uint64(11)).astype(np.float64) * (1.0 / (1 << 53))


# --------------------------------------------------------------------------
# Mesh container
# --------------------------------------------------------------------------
@dataclass
class Mesh:
    name: str
    V: np.ndarray  # [nv, 3] float64
    T: np.ndarray  # [nf, 3] int32, CCW seen from outside
    meta: dict = field(default_factory=dict)

    @property
    def nv(self) -> int:
        return int(self.V.shape[0])

    @property
    def nf(self) -> int:
        return int(self.T.shape[0])


def _finish(name, V, T, **meta) -> Mesh:
    V = np.ascontiguousarray(V, dtype=np.float64)
    T = np.ascontiguousarray(T, dtype=np.int32)
    return Mesh(name, V, T, dict(meta))


def unique_edges(T: np.ndarray) -> np.ndarray:
    e = np.concatenate([T[:, [0, 1]], T[:, [1, 2]], T[:, [2, 0]]], axis=0)
    e.sort(axis=1)
    return np.unique(e, axis=0)


def mean_edge_length(m: Mesh) -> float:
    """Mean length of the undirected edges (a workload parameter: cutoffs and
    interaction ranges of several configurations are multiples of it)."""
    e = unique_edges(m.T)
    return float(np.linalg.norm(m.V[e[:, 0]] - m.V[e[:, 1]], axis=1).mean())


def surface_area(m: Mesh) -> float:
    a = m.V[m.T[:, 1]] - m.V[m.T[:, 0]]
    b = m.V[m.T[:, 2]] - m.V[m.T[:, 0]]
    return float(0.5 * np.linalg.norm(np.cross(a, b), axis=1).sum())


def _orient_outward(V, T, center_fn):
    """Flip faces whose normal points towards ``center_fn`` of their centroid."""
    a = V[T[:, 1]] - V[T[:, 0]]
    b = V[T[:, 2]] - V[T[:, 0]]
    n = np.cross(a, b)
    c = V[T].mean(axis=1)
    out = c - center_fn(c)
    flip = (n * out).sum(axis=1) < 0
    T = T.copy()
    T[flip] = T[flip][:, [0, 2, 1]]
    return T


# --------------------------------------------------------------------------
# Closed surfaces
# --------------------------------------------------------------------------
def icosahedron() -> Mesh:
    t = (1.0 + 5.0 ** 0.5) / 2.0
    V = []
    for a in (-1.0, 1.0):
        for b in (-t, t):
            V += [(a, b, 0.0), (0.0, a, b), (b, 0.0, a)]
    V = np.array(V, dtype=np.float64)
    # faces = the 20 triples of mutually adjacent vertices (edge length 2)
    d = np.linalg.norm(V[:, None, :] - V[None, :, :], axis=2)
    adj = np.abs(d - 2.0) < 1e-9
    T = []
    for i in range(12):
        for j in range(i + 1, 12):
            if not adj[i, j]:
                continue
            for k in range(j + 1, 12):
                if adj[i, k] and adj[j, k]:
                    T.append((i, j, k))
    T = np.array(T, dtype=np.int64)
    assert T.shape == (20, 3)
    T = _orient_outward(V, T, lambda c: np.zeros_like(c))
    V = V / np.linalg.norm(V, axis=1, keepdims=True)
    return _finish("icosahedron", V, T)


def _subdivide(V, T, project):
    nv = V.shape[0]
    e = np.concatenate([T[:, [0, 1]], T[:, [1, 2]], T[:, [2, 0]]], axis=0)
    es = np.sort(e, axis=1)
    uniq, inv = np.unique(es, axis=0, return_inverse=True)
    inv = inv.reshape(-1)
    mids = project(0.5 * (V[uniq[:, 0]] + V[uniq[:, 1]]))
    nf = T.shape[0]
    m01 = nv + inv[0:nf]
    m12 = nv + inv[nf:2 * nf]
    m20 = nv + inv[2 * nf:3 * nf]
    a, b, c = T[:, 0], T[:, 1], T[:, 2]
    T2 = np.concatenate([
        np.stack([a, m01, m20], 1),
        np.stack([b, m12, m01], 1),
        np.stack([c, m20, m12], 1),
        np.stack([m01, m12, m20], 1),
    ], axis=0)
    return np.concatenate([V, mids], axis=0), T2


def icosphere(level: int, radius: float = 1.0) -> Mesh:
    """Icosahedron subdivided ``level`` times (each face into 4), midpoints
    pushed out to the sphere: level 3 has 642 vertices / 1280 faces, level 5
    10,242 / 20,480, level 6 40,962 / 81,920."""
    m = icosahedron()
    V, T = m.V, m.T.astype(np.int64)
    unit = lambda P: P / np.linalg.norm(P, axis=1, keepdims=True)
    for _ in range(level):
        V, T = _subdivide(V, T, unit)
    return _finish(f"icosphere_L{level}", radius * V, T, level=level, radius=radius)


def bumpy_sphere(level: int = 5, amp: float = 0.1) -> Mesh:
    """Icosphere whose vertices are moved radially to
    r = 1 + amp * sin(4 theta) * cos(3 phi), theta = arccos(z), phi = atan2(y, x)."""
    m = icosphere(level)
    u = m.V
    th = np.arccos(np.clip(u[:, 2], -1.0, 1.0))
    ph = np.arctan2(u[:, 1], u[:, 0])
    r = 1.0 + amp * np.sin(4.0 * th) * np.cos(3.0 * ph)
    return _finish(f"bumpy_sphere_L{level}", u * r[:, None], m.T, level=level, amp=amp)


def ellipsoid(level: int = 6, axes=(1.0, 0.8, 0.6)) -> Mesh:
    m = icosphere(level)
    return _finish(f"ellipsoid_L{level}", m.V * np.asarray(axes)[None, :], m.T, axes=tuple(axes))


def torus(R: float, r: float, n_major: int, n_minor: int) -> Mesh:
    """Tube of radius r around a circle of radius R, a regular (u, v) grid of
    n_major x n_minor quads, each split into two triangles."""
    i = np.arange(n_major)
    j = np.arange(n_minor)
    u = 2.0 * np.pi * i / n_major
    v = 2.0 * np.pi * j / n_minor
    U, W = np.meshgrid(u, v, indexing="ij")
    V = np.stack([(R + r * np.cos(W)) * np.cos(U), (R + r * np.cos(W)) * np.sin(U), r * np.sin(W)], -1).reshape(-1, 3)
    I, J = np.meshgrid(i, j, indexing="ij")
    a = (I * n_minor + J).reshape(-1)
    b = (((I + 1) % n_major) * n_minor + J).reshape(-1)
    c = (((I + 1) % n_major) * n_minor + (J + 1) % n_minor).reshape(-1)
    d = (I * n_minor + (J + 1) % n_minor).reshape(-1)
    T = np.concatenate([np.stack([a, b, c], 1), np.stack([a, c, d], 1)], 0)

    def tube_center(cpts):
        ang = np.arctan2(cpts[:, 1], cpts[:, 0])
        return np.stack([R * np.cos(ang), R * np.sin(ang), np.zeros_like(ang)], 1)

    T = _orient_outward(V, T, tube_center)
    return _finish(f"torus_{n_major}x{n_minor}", V, T, R=R, r=r, n_major=n_major, n_minor=n_minor)


def tetrahedron(edge: float = 1.0) -> Mesh:
    V = np.array([[1, 1, 1], [1, -1, -1], [-1, 1, -1], [-1, -1, 1]], dtype=np.float64)
    V *= edge / (2.0 * np.sqrt(2.0))
    T = np.array([[0, 1, 2], [0, 1, 3], [0, 2, 3], [1, 2, 3]], dtype=np.int64)
    T = _orient_outward(V, T, lambda c: np.zeros_like(c))
    return _finish("tetrahedron", V, T, edge=edge)


def cube(n: int = 1) -> Mesh:
    """Surface of the unit cube [0,1]^3, each square face an n x n grid of
    quads split into two triangles."""
    verts = {}
    Vl, Tl = [], []

    def vid(p):
        key = tuple(int(round(x * n)) for x in p)
        if key not in verts:
            verts[key] = len(Vl)
            Vl.append([k / n for k in key])
        return verts[key]

    for axis in range(3):
        for side in (0.0, 1.0):
            for a in range(n):
                for b in range(n):
                    def P(s, t):
                        p = [0.0, 0.0, 0.0]
                        p[axis] = side
                        p[(axis + 1) % 3] = s / n
                        p[(axis + 2) % 3] = t / n
                        return vid(p)
                    q = [P(a, b), P(a + 1, b), P(a + 1, b + 1), P(a, b + 1)]
                    Tl.append([q[0], q[1], q[2]])
                    Tl.append([q[0], q[2], q[3]])
    V = np.array(Vl, dtype=np.float64)
    T = np.array(Tl, dtype=np.int64)
    T = _orient_outward(V, T, lambda c: np.full_like(c, 0.5))
    return _finish(f"cube_{n}", V, T, n=n)


# --------------------------------------------------------------------------
# Open surfaces
# --------------------------------------------------------------------------
def _grid_tris(nx, ny):
    I, J = np.meshgrid(np.arange(nx), np.arange(ny), indexing="ij")
    a = (I * (ny + 1) + J).reshape(-1)
    b = ((I + 1) * (ny + 1) + J).reshape(-1)
    c = ((I + 1) * (ny + 1) + J + 1).reshape(-1)
    d = (I * (ny + 1) + J + 1).reshape(-1)
    return np.concatenate([np.stack([a, b, c], 1), np.stack([a, c, d], 1)], 0)


def flat_grid(nx: int, ny: int, sx: float = 1.0, sy: float = 1.0) -> Mesh:
    """[0,sx] x [0,sy] in the z = 0 plane, normal +z."""
    x = np.linspace(0.0, sx, nx + 1)
    y = np.linspace(0.0, sy, ny + 1)
    X, Y = np.meshgrid(x, y, indexing="ij")
    V = np.stack([X, Y, np.zeros_like(X)], -1).reshape(-1, 3)
    return _finish(f"flat_{nx}x{ny}", V, _grid_tris(nx, ny), nx=nx, ny=ny, sx=sx, sy=sy)


def corrugated_sheet(nx: int, ny: int, x0: float = 0.0, x1: float = 2 * np.pi, sy: float = 2.0) -> Mesh:
    """z = sin x sampled on a grid aligned with y: every quad is a planar
    rectangle, so the mesh develops isometrically into a flat rectangle whose
    x-side is the chord-length arc coordinate s(x)."""
    x = np.linspace(x0, x1, nx + 1)
    y = np.linspace(0.0, sy, ny + 1)
    X, Y = np.meshgrid(x, y, indexing="ij")
    V = np.stack([X, Y, np.sin(X)], -1).reshape(-1, 3)
    return _finish(f"corrugated_{nx}x{ny}", V, _grid_tris(nx, ny), nx=nx, ny=ny, x=x, sy=sy)


def height_field(n_cells: int = 316, size: float = 10.0, n_bumps: int = 40, seed: int = 2) -> Mesh:
    """z = sum of Gaussian bumps a*exp(-|(x,y)-c|^2 / (2 w^2)) over a square
    grid, every cell split along its (i,j)-(i+1,j+1) diagonal. Bump parameters
    a ~ U[0.05,0.3], w ~ U[0.1,0.5], c ~ U[0,size]^2 from SplitMix64(seed),
    drawn per bump in the order a, w, cx, cy."""
    u = uniforms(seed, 4 * n_bumps).reshape(n_bumps, 4)
    amp = 0.05 + 0.25 * u[:, 0]
    wid = 0.1 + 0.4 * u[:, 1]
    cx = size * u[:, 2]
    cy = size * u[:, 3]
    g = np.linspace(0.0, size, n_cells + 1)
    X, Y = np.meshgrid(g, g, indexing="ij")
    Z = np.zeros_like(X)
    for k in range(n_bumps):
        Z += amp[k] * np.exp(-((X - cx[k]) ** 2 + (Y - cy[k]) ** 2) / (2.0 * wid[k] ** 2))
    V = np.stack([X, Y, Z], -1).reshape(-1, 3)
    return _finish(f"heightfield_{n_cells}", V, _grid_tris(n_cells, n_cells), n_cells=n_cells, size=size,
                   bumps=np.stack([amp, wid, cx, cy], 1))


def cone_fan(theta_total: float, n: int, rho: float = 1.0) -> Mesh:
    """n congruent isosceles triangles (legs rho, apex angle theta_total/n)
    around an apex: a cone whose apex angle sum is ``theta_total``. For
    theta_total < 2 pi the rim is a planar regular n-gon below the apex; for
    theta_total > 2 pi (n even) the rim zig-zags up and down."""
    a = theta_total / (2.0 * n)
    if theta_total < 2 * np.pi:
        rr = rho * np.sin(a) / np.sin(np.pi / n)
        h = np.sqrt(max(rho * rho - rr * rr, 0.0))
        apex = np.array([0.0, 0.0, h])
        zs = np.zeros(n)
    else:
        assert n % 2 == 0
        rr = rho * np.cos(a) / np.cos(np.pi / n)
        z0 = np.sqrt(max(rho * rho - rr * rr, 0.0))
        apex = np.zeros(3)
        zs = np.array([z0 if k % 2 == 0 else -z0 for k in range(n)])
    ang = 2.0 * np.pi * np.arange(n) / n
    rim = np.stack([rr * np.cos(ang), rr * np.sin(ang), zs], 1)
    V = np.concatenate([apex[None, :], rim], 0)
    T = np.array([[0, 1 + k, 1 + (k + 1) % n] for k in range(n)], dtype=np.int64)
    return _finish(f"cone_{theta_total:.4f}_{n}", V, T, theta=theta_total, n=n, rho=rho)


def prism(n: int, R: float = 1.0, H: float = 1.0, nz: int = 2) -> Mesh:
    """Side walls of a regular n-gon prism (circumradius R, height H, open
    ends), nz rows of quads, each split into two triangles."""
    ang = 2.0 * np.pi * np.arange(n) / n
    z = np.linspace(0.0, H, nz + 1)
    V = np.array([[R * np.cos(a), R * np.sin(a), zz] for zz in z for a in ang], dtype=np.float64)
    T = []
    for r in range(nz):
        for k in range(n):
            a = r * n + k
            b = r * n + (k + 1) % n
            c = (r + 1) * n + (k + 1) % n
            d = (r + 1) * n + k
            T += [[a, b, c], [a, c, d]]
    T = np.array(T, dtype=np.int64)
    T = _orient_outward(V, T, lambda c: np.stack([np.zeros(len(c)), np.zeros(len(c)), c[:, 2]], 1))
    return _finish(f"prism_{n}", V, T, n=n, R=R, H=H, nz=nz)


def l_shape(k: int = 4) -> Mesh:
    """Flat L-shaped region [0,2]^2 minus (1,2]x(1,2], grid spacing 1/k; the
    reflex corner is at (1, 1)."""
    g = flat_grid(2 * k, 2 * k, 2.0, 2.0)
    c = g.V[g.T].mean(axis=1)
    keep = ~((c[:, 0] > 1.0) & (c[:, 1] > 1.0))
    T = g.T[keep]
    used = np.unique(T)
    remap = -np.ones(g.nv, dtype=np.int64)
    remap[used] = np.arange(len(used))
    return _finish(f"lshape_{k}", g.V[used], remap[T], k=k)


# --------------------------------------------------------------------------
# Particles
# --------------------------------------------------------------------------
def random_particles(nf: int, n: int, seed: int):
    """Face uniform over all faces, then barycentric uniform over the
    triangle: b = (1 - sqrt(u1), sqrt(u1) (1 - u2), sqrt(u1) u2). Three
    SplitMix64 draws per particle, in the order face, u1, u2."""
    u = uniforms(seed, 3 * n).reshape(n, 3)
    face = np.minimum((u[:, 0] * nf).astype(np.int64), nf - 1).astype(np.int32)
    s = np.sqrt(u[:, 1])
    bary = np.stack([1.0 - s, s * (1.0 - u[:, 2]), s * u[:, 2]], 1)
    return face, np.ascontiguousarray(bary)


# --------------------------------------------------------------------------
# Workload configurations
# --------------------------------------------------------------------------
@dataclass
class Workload:
    name: str
    mesh: Mesh
    face: np.ndarray
    bary: np.ndarray
    potential: dict
    integrator: dict
    steps: int
    mean_edge: float


C3_TORI = [(57, 17), (67, 20), (80, 24), (97, 29), (113, 34), (133, 40), (157, 47), (187, 56), (220, 66),
           (260, 78), (310, 93), (367, 110)]


def benchmark_torus() -> Mesh:
    """Torus with radii 1 and 3 (aspect ratio 3) at 83 x 28 quads, 4648
    faces: a procedural stand-in for the triangulated torus of the paper's
    scaling benchmarks (about 4600 faces)."""
    return torus(3.0, 1.0, 83, 28)


# Mesh-size sweep at fixed N (the paper's Sec. 4 study of cost against the
# number of vertices): each surface refined at fixed span, the interaction
# range one tenth of the span. Regular (u, v) tori with the quad aspect
# matched at the tube's centre line stand in for isotropic remeshing.
VSWEEP = {
    "sphere": dict(span=2.0, levels=[2, 3, 4, 5, 6]),
    "torus3": dict(span=8.0, levels=[12, 17, 24, 34, 48, 68, 96]),
    "torus20": dict(span=42.0, levels=[6, 8, 12, 17, 24, 34]),
}


def vsweep_mesh(surface: str, level: int) -> Mesh:
    """sphere: icosphere of radius 1 at `level`; torus3 / torus20: tube
    radius 1 around a circle of radius 3 / 20 with `level` quads around the
    tube and 3 / 20 times as many around the ring."""
    if surface == "sphere":
        return icosphere(level)
    if surface == "torus3":
        return torus(3.0, 1.0, 3 * level, level)
    if surface == "torus20":
        return torus(20.0, 1.0, 20 * level, level)
    raise KeyError(surface)


def packing_count(m: Mesh, sigma: float, phi: float = 0.3, lo: int = 200, hi: int = 4000) -> int:
    """Particles of diameter sigma at packing fraction phi, clamped to [lo, hi]."""
    n = int(round(phi * surface_area(m) / (np.pi * (0.5 * sigma) ** 2)))
    return int(min(max(n, lo), hi))


def workload(name: str) -> "Workload | list[Workload]":
    """The synthetic workloads:

    c1  icosphere L3 (R = 1), N = 64 (seed 0), harmonic k = 1, sigma = 0.5,
        overdamped dt = 0.01, mobility 1, 10 steps.
    c2  bumpy sphere (icosphere L5, r = 1 + 0.1 sin 4theta cos 3phi), N = 1000
        (seed 1), harmonic sigma = 0.15, overdamped, 100 steps.
    c3  16 surfaces (icospheres L3-L6 and 12 tori R = 1, r = 0.3), sigma = 2
        mean edge lengths, N at packing fraction 0.3 clamped to [200, 4000],
        seeds 100 + index, overdamped dt = 0.01 sigma^2, 50 steps.
    c4  Gaussian-bump height field on [0,10]^2 (316 x 316 cells), N = 20,000
        (seed 3), harmonic k = 1, sigma = cutoff = 3 mean edge lengths,
        Brownian kT = 0.1, friction 1, dt = 0.005, 1000 steps.
    c5a / c5b  icosphere L6 / the ellipsoid (1, 0.8, 0.6), N = 2000 (seeds
        4 / 5), Coulomb 1/r with no cutoff, FIRE, 500 iterations.
    torus_nve_<N>_<sigma>  the aspect-3 benchmark torus (4648 faces), N
        particles (seed 7), harmonic repulsion of range sigma, velocity
        Verlet (NVE) dt = 0.005, from rest.
    vsweep_<surface>_<level>  a mesh of the fixed-N sweep (VSWEEP), N = 100
        (seed 11), harmonic repulsion of range span / 10 with that cutoff,
        velocity Verlet dt = range / 200, from rest.
    quench_<k>  quench k of the crystallization study (Sec. 5): the aspect-3
        benchmark torus, N = 500 (seed 200 + k), harmonic repulsion of range
        1.2 lattice spacings of a triangular lattice of that density,
        gradient descent (overdamped, dt = 0.05 range^2), 400 steps.
    """
    if name == "c1":
        m = icosphere(3)
        f, b = random_particles(m.nf, 64, 0)
        return Workload("c1", m, f, b, dict(kind="harmonic", k=1.0, sigma=0.5, cutoff=0.5),
                        dict(kind="overdamped", dt=0.01, mobility=1.0), 10, mean_edge_length(m))
    if name == "c2":
        m = bumpy_sphere(5)
        f, b = random_particles(m.nf, 1000, 1)
        return Workload("c2", m, f, b, dict(kind="harmonic", k=1.0, sigma=0.15, cutoff=0.15),
                        dict(kind="overdamped", dt=0.01, mobility=1.0), 100, mean_edge_length(m))
    if name == "c3":
        meshes = [icosphere(lv) for lv in (3, 4, 5, 6)] + [torus(1.0, 0.3, a, b) for a, b in C3_TORI]
        out = []
        for idx, m in enumerate(meshes):
            le = mean_edge_length(m)
            sig = 2.0 * le
            n = packing_count(m, sig)
            f, b = random_particles(m.nf, n, 100 + idx)
            out.append(Workload(f"c3_{m.name}", m, f, b, dict(kind="harmonic", k=1.0, sigma=sig, cutoff=sig),
                                dict(kind="overdamped", dt=0.01 * sig * sig, mobility=1.0), 50, le))
        return out
    if name == "c4":
        m = height_field()
        le = mean_edge_length(m)
        f, b = random_particles(m.nf, 20000, 3)
        sig = 3.0 * le
        return Workload("c4", m, f, b, dict(kind="harmonic", k=1.0, sigma=sig, cutoff=sig),
                        dict(kind="brownian", dt=0.005, kT=0.1, friction=1.0, seed=3), 1000, le)
    if name.startswith("torus_nve"):
        # torus_nve_<N>_<sigma>: the NVE scaling workload on an aspect-3 torus
        _, _, n_s, sig_s = name.split("_")
        m = benchmark_torus()
        n, sig = int(n_s), float(sig_s)
        f, b = random_particles(m.nf, n, 7)
        return Workload(name, m, f, b, dict(kind="harmonic", k=1.0, sigma=sig, cutoff=sig),
                        dict(kind="verlet", dt=0.005), 100, mean_edge_length(m))
    if name.startswith("vsweep_"):
        _, surf, lv = name.split("_")
        m = vsweep_mesh(surf, int(lv))
        rng = VSWEEP[surf]["span"] / 10.0
        f, b = random_particles(m.nf, 100, 11)
        return Workload(name, m, f, b, dict(kind="harmonic", k=1.0, sigma=rng, cutoff=rng),
                        dict(kind="verlet", dt=rng / 200.0), 10, mean_edge_length(m))
    if name.startswith("quench_"):
        k = int(name.split("_")[1])
        m = benchmark_torus()
        n = 500
        f, b = random_particles(m.nf, n, 200 + k)
        a = math.sqrt(2.0 * surface_area(m) / (math.sqrt(3.0) * n))
        sig = 1.2 * a
        return Workload(name, m, f, b, dict(kind="harmonic", k=1.0, sigma=sig, cutoff=sig),
                        dict(kind="overdamped", dt=0.05 * sig * sig, mobility=1.0), 400, mean_edge_length(m))
    if name in ("c5a", "c5b"):
        m = icosphere(6) if name == "c5a" else ellipsoid(6)
        f, b = random_particles(m.nf, 2000, 4 if name == "c5a" else 5)
        le = mean_edge_length(m)
        return Workload(name, m, f, b, dict(kind="coulomb", k=1.0, sigma=1.0, cutoff=math.inf),
                        dict(kind="fire", dt=0.1 * le, max_disp=0.5 * le), 500, le)
    raise KeyError(name)
