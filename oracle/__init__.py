"""CPU FP64 oracle for the geodesic-interaction hot path (arXiv 2404.19751).

TEST INFRASTRUCTURE ONLY. Only ``tests/``, ``__graft_entry__.smoke()`` and the
benchmark's ``cpu_baseline`` leg may import this package. It shares no code
with the HIP library (``paper_2404_19751_amd``) and never calls it.

The heavy parts (mesh structure, brute-force unfolding geodesics, the shift
walk, Philox, the restricted Voronoi neighbours of Sec. 5) are plain C in
``oracle.c``; the force sum and the integrators are written here in numpy,
each following the passage it cites.
"""
from __future__ import annotations

import ctypes as C
import math
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SO = os.path.join(_HERE, "_liborc.so")

MESH_ERRORS = {1: "bad argument", 2: "non-manifold edge", 3: "inconsistent orientation",
               4: "non-manifold vertex", 5: "degenerate face"}


def build(force: bool = True) -> str:
    """Compile oracle.c with gcc (-O2, no FMA contraction, OpenMP)."""
    src = os.path.join(_HERE, "oracle.c")
    if force or not os.path.exists(_SO) or os.path.getmtime(_SO) < os.path.getmtime(src):
        tmp = _SO + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-ffp-contract=off", "-fno-fast-math", "-fopenmp", "-fPIC", "-shared",
                               "-std=c99", "-o", tmp, src, "-lm"])
        os.replace(tmp, _SO)
    return _SO


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_SO):
            build()
        L = C.CDLL(_SO)
        P = C.c_void_p
        L.orc_mesh_build.argtypes = [C.c_int, P, C.c_int, P, C.POINTER(P)]
        L.orc_mesh_build.restype = C.c_int
        L.orc_mesh_free.argtypes = [P]
        L.orc_mesh_export.argtypes = [P, P, P, P, P]
        L.orc_geodesic_pairs.argtypes = [P, C.c_int, P, P, C.c_double, C.c_int, P, C.c_int, C.c_double,
                                         C.c_double]
        L.orc_geodesic_pairs.restype = P
        L.orc_pairs_count.argtypes = [P]
        L.orc_pairs_count.restype = C.c_int64
        L.orc_pairs_tie_count.argtypes = [P]
        L.orc_pairs_tie_count.restype = C.c_int64
        L.orc_pairs_export.argtypes = [P] * 9
        L.orc_pairs_counters.argtypes = [P, P]
        L.orc_pairs_free.argtypes = [P]
        L.orc_geodesic_pairs_windows.argtypes = [P, C.c_int, P, P, C.c_double, C.c_int, P, C.c_int]
        L.orc_geodesic_pairs_windows.restype = P
        L.orc_pairs_window_counters.argtypes = [P, P]
        L.orc_walk.argtypes = [P, C.c_int, P, P, P, P, P, P]
        L.orc_walk.restype = C.c_int
        L.orc_philox4x32_10.argtypes = [P, P, P]
        L.orc_voronoi_pairs.argtypes = [P, C.c_int, P, C.c_double, P]
        L.orc_voronoi_pairs.restype = C.c_int
        _lib = L
    return _lib


def _p(a):
    return a.ctypes.data_as(C.c_void_p)


class OracleMesh:
    """Half-edge mesh built by the oracle's own code."""

    def __init__(self, V, T):
        self.V = np.ascontiguousarray(V, dtype=np.float64)
        self.T = np.ascontiguousarray(T, dtype=np.int32)
        h = C.c_void_p()
        rc = lib().orc_mesh_build(self.V.shape[0], _p(self.V), self.T.shape[0], _p(self.T), C.byref(h))
        if rc != 0:
            raise ValueError(f"oracle mesh rejected: {MESH_ERRORS.get(rc, rc)}")
        self._h = h
        nv, nf = self.V.shape[0], self.T.shape[0]
        self.twin = np.empty(3 * nf, np.int32)
        self.theta = np.empty(nv, np.float64)
        self.pseudo = np.empty(nv, np.uint8)
        self.boundary = np.empty(nv, np.uint8)
        lib().orc_mesh_export(h, _p(self.twin), _p(self.theta), _p(self.pseudo), _p(self.boundary))
        a = self.V[self.T[:, 1]] - self.V[self.T[:, 0]]
        b = self.V[self.T[:, 2]] - self.V[self.T[:, 0]]
        n = np.cross(a, b)
        self.area2 = np.linalg.norm(n, axis=1)
        self.normal = n / self.area2[:, None]
        self.ex = a / np.linalg.norm(a, axis=1, keepdims=True)
        self.ey = np.cross(self.normal, self.ex)

    def __del__(self):
        try:
            if getattr(self, "_h", None):
                lib().orc_mesh_free(self._h)
                self._h = None
        except Exception:
            pass

    def xyz(self, face, bary):
        return np.einsum("nk,nkd->nd", bary, self.V[self.T[face]])


class Pairs:
    def __init__(self, off, nbr, dist, tan, flags, tie_off, tie_tan, tie_dist, counters, tie_rel, cone_slack):
        self.off, self.nbr, self.dist, self.tan, self.flags = off, nbr, dist, tan, flags
        self.tie_off, self.tie_tan, self.tie_dist = tie_off, tie_tan, tie_dist
        self.counters, self.tie_rel, self.cone_slack = counters, tie_rel, cone_slack

    def ties(self, p):
        """Initial directions of the pair's tie set."""
        return self.tie_tan[self.tie_off[p]:self.tie_off[p + 1]]

    def tie_lengths(self, p):
        """Length of the shortest path found in each direction of ties(p)."""
        return self.tie_dist[self.tie_off[p]:self.tie_off[p + 1]]


def geodesic_pairs(mesh: OracleMesh, face, bary, cutoff, sources=None, nthreads=0, tie_rel=1e-9,
                   cone_slack=0.0) -> Pairs:
    """Exact geodesic distances d_ij < cutoff and initial unit tangents t_ij
    (3D, in the plane of the source's face) for every source i (Sec. 3.1:
    lengths l_ij and tangents relative to the source; submeshing by the
    Euclidean lower bound). ``cutoff = inf`` asks for all pairs.

    Where several shortest paths leave the source in different directions
    (the cut locus), the tangent is not unique: ``ties(p)`` lists the
    initial direction of every path within ``tie_rel * d`` of the shortest
    (1e-9 by default; the FP32-mixed comparisons use 1e-5, their distance
    tolerance), and such a pair is flagged (bit 0).

    ``cone_slack`` (the sine of an angle; 0 means exact cones up to 1e-12)
    widens the test of whether a target lies in a straight link's cone, so
    that the tie set also holds the directions of straight links to points
    within that angle of the target: the resolution of a computation in
    reduced precision, whose cone tests are perturbed by its rounding. The
    reported distance then may fall short of the exact one by a term of
    second order in that angle."""
    face = np.ascontiguousarray(face, np.int32)
    bary = np.ascontiguousarray(bary, np.float64)
    src = None if sources is None else np.ascontiguousarray(sources, np.int32)
    nsrc = face.shape[0] if src is None else src.shape[0]
    L = lib()
    h = L.orc_geodesic_pairs(mesh._h, face.shape[0], _p(face), _p(bary), float(cutoff if math.isfinite(cutoff) else -1.0),
                             nsrc, None if src is None else _p(src), int(nthreads), float(tie_rel),
                             float(cone_slack))
    if not h:
        raise ValueError("oracle rejected the particle state")
    try:
        P = L.orc_pairs_count(h)
        Tn = L.orc_pairs_tie_count(h)
        off = np.empty(nsrc + 1, np.int64)
        nbr = np.empty(P, np.int32)
        dist = np.empty(P, np.float64)
        tan = np.empty((P, 3), np.float64)
        flags = np.empty(P, np.uint8)
        tie_off = np.empty(P + 1, np.int64)
        tie_tan = np.empty((Tn, 3), np.float64)
        tie_dist = np.empty(Tn, np.float64)
        L.orc_pairs_export(h, _p(off), _p(nbr), _p(dist), _p(tan), _p(flags), _p(tie_off), _p(tie_tan), _p(tie_dist))
        cnt = np.empty(5, np.int64)
        L.orc_pairs_counters(h, _p(cnt))
    finally:
        L.orc_pairs_free(h)
    return Pairs(off, nbr, dist, tan, flags, tie_off, tie_tan, tie_dist,
                 dict(windows=int(cnt[0]), pruned=int(cnt[1]), roots=int(cnt[2]), improvements=int(cnt[3]),
                      rejected=int(cnt[4])), float(tie_rel), float(cone_slack))


def geodesic_pairs_windows(mesh: OracleMesh, face, bary, cutoff, sources=None, nthreads=0) -> Pairs:
    """The pairs of ``geodesic_pairs`` by the exact window-propagation method
    of Sec. 2.2 (MMP's continuous Dijkstra: windows on half-edges, processed
    in distance order, trimmed to the pointwise minimum on every edge;
    pseudo-source vertices launched once). An independent route to the same
    distances, and the method's own work count: ``counters`` holds windows
    inserted, propagated and trimmed, pseudo-source launches, faces entered,
    insertions dropped and sources rejected. One direction per pair (no tie
    sets; the tie flag is never set)."""
    face = np.ascontiguousarray(face, np.int32)
    bary = np.ascontiguousarray(bary, np.float64)
    src = None if sources is None else np.ascontiguousarray(sources, np.int32)
    nsrc = face.shape[0] if src is None else src.shape[0]
    L = lib()
    h = L.orc_geodesic_pairs_windows(mesh._h, face.shape[0], _p(face), _p(bary),
                                     float(cutoff if math.isfinite(cutoff) else -1.0), nsrc,
                                     None if src is None else _p(src), int(nthreads))
    if not h:
        raise ValueError("oracle rejected the particle state")
    try:
        P = L.orc_pairs_count(h)
        off = np.empty(nsrc + 1, np.int64)
        nbr = np.empty(P, np.int32)
        dist = np.empty(P, np.float64)
        tan = np.empty((P, 3), np.float64)
        flags = np.empty(P, np.uint8)
        tie_off = np.empty(P + 1, np.int64)
        tie_tan = np.empty((P, 3), np.float64)
        tie_dist = np.empty(P, np.float64)
        L.orc_pairs_export(h, _p(off), _p(nbr), _p(dist), _p(tan), _p(flags), _p(tie_off), _p(tie_tan), _p(tie_dist))
        cnt = np.empty(7, np.int64)
        L.orc_pairs_window_counters(h, _p(cnt))
    finally:
        L.orc_pairs_free(h)
    names = ("inserted", "propagated", "trimmed", "launches", "faces", "dropped", "rejected")
    return Pairs(off, nbr, dist, tan, flags, tie_off, tie_tan, tie_dist,
                 {k: int(v) for k, v in zip(names, cnt)}, 0.0, 0.0)


def walk(mesh: OracleMesh, face, bary, disp, vel=None):
    """The shift walk (Sec. 3.2): returns new (face, bary, vel, stats, flags)."""
    face = np.array(face, np.int32, copy=True)
    bary = np.array(bary, np.float64, copy=True)
    disp = np.ascontiguousarray(disp, np.float64)
    v = None if vel is None else np.array(vel, np.float64, copy=True)
    st = np.zeros(5, np.int64)
    fl = np.zeros(face.shape[0], np.uint8)
    lib().orc_walk(mesh._h, face.shape[0], _p(face), _p(bary), _p(disp), None if v is None else _p(v), _p(st), _p(fl))
    stats = dict(crossings=int(st[0]), vertex_hits=int(st[1]), boundary_hits=int(st[2]), cap_hits=int(st[3]),
                 near_vertex=int(st[4]))
    return face, bary, v, stats, fl


# --------------------------------------------------------------------------
# Potentials and the force sum (Sec. 2.1 Gaussian example; Sec. 3.1 force sum)
# --------------------------------------------------------------------------
def potential(kind, d, k=1.0, sigma=1.0):
    """U(d) and dU/dd.
    harmonic U = (k/2)(1 - d/sigma)^2 for d < sigma, else 0;
    coulomb  U = k/d;
    gaussian U = k exp(-d^2 / (2 sigma^2)) (Sec. 2.1)."""
    d = np.asarray(d, np.float64)
    if kind == "harmonic":
        x = 1.0 - d / sigma
        inside = d < sigma
        U = np.where(inside, 0.5 * k * x * x, 0.0)
        dU = np.where(inside, -(k / sigma) * x, 0.0)
    elif kind == "coulomb":
        U = k / d
        dU = -k / (d * d)
    elif kind == "gaussian":
        U = k * np.exp(-d * d / (2.0 * sigma * sigma))
        dU = -(d / (sigma * sigma)) * U
    else:
        raise KeyError(kind)
    return U, dU


def forces(n, pairs: Pairs, kind, k=1.0, sigma=1.0):
    """F_i = sum_j U'(d_ij) t_ij (the force sum of Sec. 3.1, with t_ij the unit
    tangent at i pointing towards j, so a repulsive U' < 0 pushes i away from
    j); E = (1/2) sum_i sum_j U(d_ij). Pairs at zero distance are skipped.
    Plain FP64 sums in ascending j."""
    F = np.zeros((n, 3))
    E = 0.0
    for i in range(n):
        a, b = pairs.off[i], pairs.off[i + 1]
        for p in range(a, b):
            d = pairs.dist[p]
            if d <= 0.0:
                continue
            U, dU = potential(kind, d, k, sigma)
            F[i] += float(dU) * pairs.tan[p]
            E += 0.5 * float(U)
    return F, E


# --------------------------------------------------------------------------
# Integrators (Sec. 2.1: overdamped / Brownian dynamics)
# --------------------------------------------------------------------------
def philox4x32_10(ctr, key):
    c = (C.c_uint32 * 4)(*[int(x) & 0xFFFFFFFF for x in ctr])
    k = (C.c_uint32 * 2)(*[int(x) & 0xFFFFFFFF for x in key])
    o = (C.c_uint32 * 4)()
    lib().orc_philox4x32_10(C.cast(c, C.c_void_p), C.cast(k, C.c_void_p), C.cast(o, C.c_void_p))
    return [int(x) for x in o]


def gaussian_pair(seed: int, step: int, particle: int):
    """Two standard normals for (step, particle): Philox4x32-10 with counter
    (particle, step lo, step hi, 0) and key (seed lo, seed hi); the four words
    make two 53-bit uniforms u1, u2 (top 27 + 26 bits), and Box-Muller gives
    (r cos 2 pi u2, r sin 2 pi u2) with r = sqrt(-2 ln(1 - u1))."""
    w = philox4x32_10([particle, step & 0xFFFFFFFF, (step >> 32) & 0xFFFFFFFF, 0],
                      [seed & 0xFFFFFFFF, (seed >> 32) & 0xFFFFFFFF])
    u1 = ((w[0] >> 5) * 67108864.0 + (w[1] >> 6)) * (1.0 / 9007199254740992.0)
    u2 = ((w[2] >> 5) * 67108864.0 + (w[3] >> 6)) * (1.0 / 9007199254740992.0)
    r = math.sqrt(-2.0 * math.log(1.0 - u1))
    return r * math.cos(2.0 * math.pi * u2), r * math.sin(2.0 * math.pi * u2)


def displacement(mesh: OracleMesh, face, F, integ: dict, step: int = 0):
    """Displacement D_i for one step.
    overdamped:  D = mobility dt F;
    brownian:    friction D = dt F + sqrt(2 kT friction dt) (eta1 ex + eta2 ey)
                 (the discrete Brownian update of Sec. 2.1, one unit normal per
                 tangent-plane axis of the particle's face)."""
    kind = integ["kind"]
    if kind == "overdamped":
        return integ.get("mobility", 1.0) * integ["dt"] * F
    if kind == "brownian":
        lam, dt, kT, seed = integ.get("friction", 1.0), integ["dt"], integ["kT"], int(integ.get("seed", 0))
        amp = math.sqrt(2.0 * kT * lam * dt)
        D = (dt / lam) * F
        for i in range(F.shape[0]):
            e1, e2 = gaussian_pair(seed, step, i)
            D[i] += (amp / lam) * (e1 * mesh.ex[face[i]] + e2 * mesh.ey[face[i]])
        return D
    raise KeyError(kind)


def step(mesh: OracleMesh, face, bary, potential_cfg: dict, integ: dict, step_index: int = 0, nthreads=0):
    """One full step: pairs -> forces -> displacement -> walk."""
    pr = geodesic_pairs(mesh, face, bary, potential_cfg["cutoff"], nthreads=nthreads)
    F, E = forces(face.shape[0], pr, potential_cfg["kind"], potential_cfg.get("k", 1.0), potential_cfg.get("sigma", 1.0))
    D = displacement(mesh, face, F, integ, step_index)
    f2, b2, _, st, fl = walk(mesh, face, bary, D)
    return f2, b2, dict(pairs=pr, F=F, E=E, D=D, walk=st, walk_flags=fl)


# --------------------------------------------------------------------------
# FIRE energy minimisation (Bitzek, Koskinen, Gähler, Moseler & Gumbsch,
# "Structural relaxation made simple", Phys. Rev. Lett. 97, 170201 (2006))
# --------------------------------------------------------------------------
FIRE_DEFAULTS = dict(alpha0=0.1, f_alpha=0.99, f_inc=1.1, f_dec=0.5, n_min=5)


def fire_init(integ: dict) -> dict:
    """FIRE state before the first iteration: time step dt0 = integ["dt"],
    mixing factor alpha0, no iteration with positive power yet."""
    p = dict(FIRE_DEFAULTS)
    p.update({k: integ[k] for k in FIRE_DEFAULTS if k in integ})
    return dict(dt=float(integ["dt"]), alpha=float(p["alpha0"]), n_pos=0)


def fire_step(mesh: OracleMesh, face, bary, vel, potential_cfg: dict, integ: dict, state: dict, nthreads=0):
    """One FIRE iteration on the surface, with unit masses.

    With F the forces at the current positions and P = sum_i F_i . v_i:
      P > 0:  v <- (1 - alpha) v + alpha |v| F / |F|  (norms over all
              particles); after more than n_min consecutive such iterations
              dt <- min(f_inc dt, dt_max) and alpha <- f_alpha alpha;
      P <= 0: v <- 0, dt <- f_dec dt, alpha <- alpha0.
    Then the semi-implicit Euler step v <- v + dt F, and each particle walks
    the displacement D_i = dt v_i (capped at max_disp in length) along the
    surface, its velocity parallel-transported by the walk. dt_max defaults
    to 10 dt0 and max_disp to infinity.
    Returns (face, bary, vel, state, info)."""
    p = dict(FIRE_DEFAULTS)
    p.update({k: integ[k] for k in FIRE_DEFAULTS if k in integ})
    dt_max = float(integ.get("dt_max", 10.0 * integ["dt"]))
    max_disp = float(integ.get("max_disp", math.inf))
    pr = geodesic_pairs(mesh, face, bary, potential_cfg["cutoff"], nthreads=nthreads)
    F, E = forces(face.shape[0], pr, potential_cfg["kind"], potential_cfg.get("k", 1.0),
                  potential_cfg.get("sigma", 1.0))
    v = np.array(vel, np.float64, copy=True)
    dt, alpha, n_pos = state["dt"], state["alpha"], state["n_pos"]
    P = float(np.sum(F * v))
    if P > 0.0:
        vn = math.sqrt(float(np.sum(v * v)))
        fn = math.sqrt(float(np.sum(F * F)))
        if fn > 0.0:
            v = (1.0 - alpha) * v + (alpha * vn / fn) * F
        n_pos += 1
        if n_pos > p["n_min"]:
            dt = min(dt * p["f_inc"], dt_max)
            alpha *= p["f_alpha"]
    else:
        v[:] = 0.0
        dt *= p["f_dec"]
        alpha = p["alpha0"]
        n_pos = 0
    v = v + dt * F
    D = dt * v
    L = np.linalg.norm(D, axis=1)
    over = L > max_disp
    D[over] *= (max_disp / L[over])[:, None]
    f2, b2, v2, st, fl = walk(mesh, face, bary, D, v)
    new_state = dict(dt=dt, alpha=alpha, n_pos=n_pos)
    return f2, b2, v2, new_state, dict(pairs=pr, F=F, E=E, D=D, P=P, walk=st, walk_flags=fl)


# --------------------------------------------------------------------------
# Velocity Verlet (Sec. 2.1: Newton's equation, Eq. (1); the integrator of the
# paper's NVE benchmark, Sec. 4) in leapfrog form, unit masses
# --------------------------------------------------------------------------
def verlet_step(mesh: OracleMesh, face, bary, vel, potential_cfg: dict, integ: dict, nthreads=0):
    """One step of velocity Verlet in leapfrog form on the surface. The
    velocity carried between steps is the half-step velocity v_{k-1/2}:
      v_{k+1/2} = v_{k-1/2} + dt F(x_k),   x_{k+1} = x_k walked by dt v_{k+1/2},
    the velocity parallel-transported by the walk (the kick and the drift of
    two successive half steps combined). The velocity at step k is
    v_k = v_{k-1/2} + (dt/2) F(x_k). Returns (face, bary, vel, info)."""
    pr = geodesic_pairs(mesh, face, bary, potential_cfg["cutoff"], nthreads=nthreads)
    F, E = forces(face.shape[0], pr, potential_cfg["kind"], potential_cfg.get("k", 1.0),
                  potential_cfg.get("sigma", 1.0))
    dt = float(integ["dt"])
    v = np.array(vel, np.float64, copy=True) + dt * F
    f2, b2, v2, st, fl = walk(mesh, face, bary, dt * v, v)
    return f2, b2, v2, dict(pairs=pr, F=F, E=E, walk=st, walk_flags=fl)


def positions(mesh: OracleMesh, face, bary):
    """3D points of (face, barycentric) positions: the barycentric
    combination of the face's vertices (Sec. 3.2 particle state)."""
    T = mesh.T[np.asarray(face)]
    return np.einsum("ik,ikd->id", np.asarray(bary, np.float64), mesh.V[T])


def voronoi_neighbours(mesh: OracleMesh, face, bary, tol_rel=1e-10):
    """Restricted Voronoi neighbours of the particles on the surface (Sec. 5,
    the in-surface Voronoi diagram from which the paper counts each
    particle's neighbours): a boolean n x n adjacency matrix. Two particles
    are neighbours when the surface points equidistant (3D) from both and no
    farther from either than from any other particle form a set longer than
    tol_rel times the mean edge length."""
    xyz = np.ascontiguousarray(positions(mesh, face, bary))
    n = len(xyz)
    adj = np.zeros((n, n), np.uint8)
    lbar = float(np.mean(np.linalg.norm(mesh.V[mesh.T[:, [1, 2, 0]]] - mesh.V[mesh.T], axis=2)))
    rc = lib().orc_voronoi_pairs(mesh._h, n, _p(xyz), tol_rel * lbar, _p(adj))
    if rc:
        raise ValueError("bad argument")
    return adj.astype(bool)

