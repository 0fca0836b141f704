"""GPU parity of the all-pairs path (no cutoff: every other particle is a
neighbour) and of the FIRE integrator, against the CPU oracle.

Small meshes of every kind (closed convex, closed with saddles, open with a
boundary, a cone apex) are compared over all pairs; the long-range
workloads (icosphere level 6 and the ellipsoid, N = 2000) are compared on
sampled source rows, with the whole launch run at full size."""
import math
import sys
import time

import numpy as np
import pytest

from paper_2404_19751_amd import workloads as W
from tests.test_gpu_fp32 import compare32
from tests.test_gpu_parity import compare_pairs
from tests.util import oracle_band

pytestmark = pytest.mark.gpu
# sampled source rows of the N = 2000 all-pairs workloads: 64 sources spread
# over the whole index range (the first and the last included)
C5_ROWS = np.unique(np.linspace(0, 1999, 64).round().astype(np.int32))


def log(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _ctx(prec):
    from paper_2404_19751_amd import gsim
    return gsim.Context(0, prec)


SMALL = [
    ("icosphere3", lambda: W.icosphere(3), 64),
    ("torus", lambda: W.torus(1.0, 0.3, 30, 12), 60),
    ("bumpy_l2", lambda: W.bumpy_sphere(2, 0.15), 50),
    ("lshape", lambda: W.l_shape(4), 40),
    ("cone_saddle", lambda: W.cone_fan(2.5 * np.pi, 8), 30),
    ("cube", lambda: W.cube(3), 40),
]


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
@pytest.mark.parametrize("name,mk,n", SMALL)
def test_allpairs_small(orc, name, mk, n, prec):
    m = mk()
    f, b = W.random_particles(m.nf, n, 23)
    ctx = _ctx(prec)
    try:
        mid = ctx.mesh_upload(m.V, m.T)
        ctx.particles_set(mid, f, b)
        log(f"[gpu-all] {name} {prec}: all pairs of {n}")
        g = ctx.geodesic_pairs(mid, math.inf)
        cnt = ctx.counters()
        assert cnt["limited"] == 0, cnt
        o = orc.geodesic_pairs(orc.OracleMesh(m.V, m.T), f, b, math.inf, **oracle_band(prec))
        assert len(o.dist) == n * (n - 1)
        if prec == "fp64":
            err = compare_pairs(g, o, W.mean_edge_length(m), label=name)
        else:
            err, _ = compare32(g, o, W.mean_edge_length(m), name)
        log(f"[gpu-all] {name} {prec}: err {err:.2e} windows {cnt['windows']}")
    finally:
        ctx.close()


MANY_SADDLES = [
    ("bumpy_l3", lambda: W.bumpy_sphere(3, 0.15), 40),
    ("torus_a3", lambda: W.torus(3.0, 1.0, 48, 16), 40),
]


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
@pytest.mark.parametrize("name,mk,n", MANY_SADDLES)
def test_allpairs_many_bend_vertices(orc, name, mk, n, prec):
    """Whole-mesh propagation on surfaces with hundreds of saddle vertices
    (every one of them a bend vertex that a source's front reaches): all
    pairs against the oracle."""
    m = mk()
    f, b = W.random_particles(m.nf, n, 29)
    ctx = _ctx(prec)
    try:
        mid = ctx.mesh_upload(m.V, m.T)
        npseudo = ctx.mesh_info(mid)["n_pseudo_sources"]
        assert npseudo > 255
        ctx.particles_set(mid, f, b)
        log(f"[gpu-all] {name} {prec}: all pairs of {n}, {npseudo} bend vertices")
        g = ctx.geodesic_pairs(mid, math.inf)
        cnt = ctx.counters()
        assert cnt["limited"] == 0, cnt
        o = orc.geodesic_pairs(orc.OracleMesh(m.V, m.T), f, b, math.inf, **oracle_band(prec))
        if prec == "fp64":
            err = compare_pairs(g, o, W.mean_edge_length(m), label=name)
        else:
            err, _ = compare32(g, o, W.mean_edge_length(m), name)
        log(f"[gpu-all] {name} {prec}: err {err:.2e} windows {cnt['windows']} launches {cnt['launches']}")
    finally:
        ctx.close()


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
@pytest.mark.parametrize("name", ["c5a", "c5b"])
def test_c5_sampled_rows(orc, name, prec):
    """Full-size all-pairs launch (N = 2000 on 81,920 faces); the rows of 64
    sampled sources against the oracle's rows for the same sources."""
    w = W.workload(name)
    ctx = _ctx(prec)
    try:
        mid = ctx.mesh_upload(w.mesh.V, w.mesh.T)
        ctx.particles_set(mid, w.face, w.bary)
        log(f"[gpu-all] {name} {prec}: all pairs of {len(w.face)} on {w.mesh.nf} faces")
        t0 = time.perf_counter()
        g = ctx.geodesic_pairs(mid, math.inf)
        dt = time.perf_counter() - t0
        cnt = ctx.counters()
        log(f"[gpu-all] {name} {prec}: {len(g['dist'])} pairs in {dt:.3f} s, counters {cnt}")
        assert cnt["limited"] == 0
        n = len(w.face)
        assert len(g["dist"]) == n * (n - 1)
        srcs = C5_ROWS
        o = orc.geodesic_pairs(orc.OracleMesh(w.mesh.V, w.mesh.T), w.face, w.bary, math.inf, sources=srcs,
                               **oracle_band(prec))
        # the GPU rows of the sampled sources, as a pairs structure of their own
        sub = {"off": [0], "nbr": [], "dist": [], "tan": [], "flags": []}
        for i in srcs:
            a, bb = g["off"][i], g["off"][i + 1]
            for key in ("nbr", "dist", "tan", "flags"):
                sub[key].append(g[key][a:bb])
            sub["off"].append(sub["off"][-1] + bb - a)
        gs = {k: (np.concatenate(v) if k != "off" else np.array(v, np.int64)) for k, v in sub.items()}
        if prec == "fp64":
            err = compare_pairs(gs, o, w.mean_edge, label=name)
        else:
            err, _ = compare32(gs, o, w.mean_edge, name)
        log(f"[gpu-all] {name} {prec}: sampled rows err {err:.2e}")
    finally:
        ctx.close()


def test_coulomb_forces_all_pairs(orc):
    """Coulomb forces over all pairs (no cutoff) on a small sphere."""
    from paper_2404_19751_amd import gsim
    m = W.icosphere(3)
    f, b = W.random_particles(m.nf, 48, 31)
    ctx = _ctx("fp64")
    try:
        mid = ctx.mesh_upload(m.V, m.T)
        ctx.particles_set(mid, f, b)
        F, E = ctx.compute_forces(mid, gsim.potential("coulomb", 1.0, 1.0, math.inf))
        o = orc.geodesic_pairs(orc.OracleMesh(m.V, m.T), f, b, math.inf)
        Fo, Eo = orc.forces(48, o, "coulomb", 1.0, 1.0)
        scale = np.zeros(48)
        for i in range(48):
            scale[i] = np.sum(1.0 / o.dist[o.off[i]:o.off[i + 1]] ** 2)
        assert np.all(np.linalg.norm(F - Fo, axis=1) <= 1e-11 * scale)
        assert abs(E - Eo) <= 1e-11 * abs(Eo)
    finally:
        ctx.close()


@pytest.mark.parametrize("mesh_name,n,iters", [("icosphere3", 32, 6), ("torus", 40, 4)])
def test_fire_iterations(orc, mesh_name, n, iters):
    """FIRE iterations (Coulomb, all pairs) on the GPU against the oracle's,
    one at a time from the same state (stage parity: faces bit-exact,
    barycentrics and velocities within 1e-10)."""
    from paper_2404_19751_amd import gsim
    m = dict(SMALL_MESHES)[mesh_name]()
    om = orc.OracleMesh(m.V, m.T)
    f, b = W.random_particles(m.nf, n, 41)
    le = W.mean_edge_length(m)
    ig_o = dict(kind="fire", dt=0.05, max_disp=0.5 * le)
    pot_o = dict(kind="coulomb", k=1.0, sigma=1.0, cutoff=math.inf)
    ctx = _ctx("fp64")
    try:
        mid = ctx.mesh_upload(m.V, m.T)
        ctx.particles_set(mid, f, b)
        pot = gsim.potential("coulomb", 1.0, 1.0, math.inf)
        ig = gsim.integrator("fire", 0.05, max_disp=0.5 * le)
        st = orc.fire_init(ig_o)
        v = np.zeros((n, 3))
        for it in range(iters):
            ctx.step(mid, pot, ig, 1)
            f, b, v, st, info = orc.fire_step(om, f, b, v, pot_o, ig_o, st)
            fg, bg, vg, _ = ctx.particles_get(mid)
            ok = info["walk_flags"] & 3 == 0
            assert np.array_equal(fg[ok], f[ok]), f"iteration {it}: faces differ"
            assert np.abs(bg[ok] - b[ok]).max() < 1e-10, f"iteration {it}"
            assert np.abs(vg[ok] - v[ok]).max() < 1e-10 * max(1.0, np.abs(v).max()), f"iteration {it}"
            # continue both from the GPU state (stage parity); setting the
            # particles restarts the GPU's FIRE state, so the oracle restarts too
            f, b, v = fg, bg, vg
            ctx.particles_set(mid, f, b, v)
            st = orc.fire_init(ig_o)
        log(f"[gpu-all] FIRE {mesh_name}: {iters} iterations match")
    finally:
        ctx.close()


def test_fire_state_carries_over(orc):
    """Several FIRE iterations in one call (the device-side dt / alpha /
    counter state carried from iteration to iteration) against the oracle's
    sequence."""
    from paper_2404_19751_amd import gsim
    m = W.icosphere(3)
    om = orc.OracleMesh(m.V, m.T)
    n = 24
    f, b = W.random_particles(m.nf, n, 43)
    le = W.mean_edge_length(m)
    ig_o = dict(kind="fire", dt=0.05, max_disp=0.5 * le)
    pot_o = dict(kind="coulomb", k=1.0, sigma=1.0, cutoff=math.inf)
    ctx = _ctx("fp64")
    try:
        mid = ctx.mesh_upload(m.V, m.T)
        ctx.particles_set(mid, f, b)
        ctx.step(mid, gsim.potential("coulomb", 1.0, 1.0, math.inf), gsim.integrator("fire", 0.05, max_disp=0.5 * le), 8)
        st = orc.fire_init(ig_o)
        v = np.zeros((n, 3))
        flags = np.zeros(n, np.int64)
        for it in range(8):
            f, b, v, st, info = orc.fire_step(om, f, b, v, pot_o, ig_o, st)
            flags |= info["walk_flags"]
        fg, bg, vg, _ = ctx.particles_get(mid)
        ok = flags & 3 == 0
        assert ok.mean() > 0.9
        assert np.array_equal(fg[ok], f[ok])
        assert np.abs(bg[ok] - b[ok]).max() < 1e-9
    finally:
        ctx.close()


SMALL_MESHES = [("icosphere3", lambda: W.icosphere(3)), ("torus", lambda: W.torus(1.0, 0.3, 30, 12))]


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_allpairs_5000_particles(orc, prec):
    """More particles than a target table in LDS could hold (the table lives
    in global memory): 5000 particles on the level-4 icosphere, 24,995,000
    pairs in one launch; sampled rows, including sources and targets with
    indices beyond 4096, against the oracle."""
    m = W.icosphere(4)
    f, b = W.random_particles(m.nf, 5000, 11)
    ctx = _ctx(prec)
    try:
        mid = ctx.mesh_upload(m.V, m.T)
        ctx.particles_set(mid, f, b)
        log(f"[gpu-all] icosphere4 n=5000 {prec}: all pairs")
        g = ctx.geodesic_pairs(mid, math.inf)
        cnt = ctx.counters()
        log(f"[gpu-all] icosphere4 n=5000 {prec}: {len(g['dist'])} pairs, counters {cnt}")
        assert cnt["limited"] == 0
        assert len(g["dist"]) == 5000 * 4999
        srcs = np.array([0, 4100, 4999], np.int32)
        o = orc.geodesic_pairs(orc.OracleMesh(m.V, m.T), f, b, math.inf, sources=srcs, **oracle_band(prec))
        sub = {"off": [0], "nbr": [], "dist": [], "tan": [], "flags": []}
        for i in srcs:
            a, bb = g["off"][i], g["off"][i + 1]
            for key in ("nbr", "dist", "tan", "flags"):
                sub[key].append(g[key][a:bb])
            sub["off"].append(sub["off"][-1] + bb - a)
        gs = {k: (np.concatenate(v) if k != "off" else np.array(v, np.int64)) for k, v in sub.items()}
        if prec == "fp64":
            err = compare_pairs(gs, o, W.mean_edge_length(m), label="icosphere4 n=5000")
        else:
            err, _ = compare32(gs, o, W.mean_edge_length(m), "icosphere4 n=5000")
        log(f"[gpu-all] icosphere4 n=5000 {prec}: sampled rows err {err:.2e}")
    finally:
        ctx.close()
