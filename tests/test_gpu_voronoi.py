"""GPU parity of the in-surface Voronoi neighbours (Sec. 5) against the
oracle: the adjacency is an integer result, compared exactly, on random
particles over several surfaces, on configurations whose neighbours are
fixed by symmetry, and on a quenched (locally relaxed) torus crystal."""
import sys

import numpy as np
import pytest

from paper_2404_19751_amd import workloads as W
from tests.util import place

pytestmark = pytest.mark.gpu


def log(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def gpu_adjacency(ctx, mid, n):
    off, nbr = ctx.voronoi_neighbours(mid)
    adj = np.zeros((n, n), bool)
    for i in range(n):
        row = nbr[off[i]:off[i + 1]]
        assert np.all(np.diff(row) > 0)
        adj[i, row] = True
    return adj


CASES = [
    ("torus_a3", W.benchmark_torus, 500, 91),
    ("sphere_l4", lambda: W.icosphere(4), 300, 93),
    ("bumpy_sphere", lambda: W.bumpy_sphere(5), 1000, 95),
    ("torus_a20", lambda: W.torus(20.0, 1.0, 240, 12), 300, 97),
    ("height_field", lambda: W.height_field(60, 10.0, 10, 2), 400, 99),
]


@pytest.mark.parametrize("name,mk,n,seed", CASES)
def test_voronoi_matches_oracle(orc, name, mk, n, seed):
    from paper_2404_19751_amd import gsim
    m = mk()
    f, b = W.random_particles(m.nf, n, seed)
    ctx = gsim.Context(0, "fp64")
    try:
        mid = ctx.mesh_upload(m.V, m.T)
        ctx.particles_set(mid, f, b)
        log(f"[gpu-voronoi] {name}: {n} particles on {m.nf} faces")
        g = gpu_adjacency(ctx, mid, n)
    finally:
        ctx.close()
    o = orc.voronoi_neighbours(orc.OracleMesh(m.V, m.T), f, b)
    assert np.array_equal(g, o), f"{name}: {int((g != o).sum())} adjacency entries differ"
    z = g.sum(1)
    log(f"[gpu-voronoi] {name}: coordination min {z.min()} mean {z.mean():.3f} max {z.max()}")


def test_voronoi_symmetric_configurations():
    from paper_2404_19751_amd import gsim
    ctx = gsim.Context(0, "fp64")
    try:
        m = W.icosphere(3)
        # the 12 icosahedron vertices, each moved 1e-4 of the way into a face
        # (particles may not sit exactly on a mesh vertex); the neighbours of
        # the icosahedron do not change under so small a move
        pts = []
        for k in range(12):
            fk = int(np.nonzero((m.T == k).any(1))[0][0])
            pts.append(m.V[k] + 1e-4 * (m.V[m.T[fk]].mean(0) - m.V[k]))
        f, b = place(m, np.array(pts))
        mid = ctx.mesh_upload(m.V, m.T)
        ctx.particles_set(mid, f, b)
        assert (gpu_adjacency(ctx, mid, 12).sum(1) == 5).all()
        c = W.cube(3)
        lo, hi = c.V.min(0), c.V.max(0)
        cen, h = 0.5 * (lo + hi), 0.5 * (hi - lo)
        pts = []
        for ax in range(3):
            for sgn in (1.0, -1.0):
                p = cen.copy()
                p[ax] += sgn * h[ax]
                pts.append(p)
        f, b = place(c, pts)
        mid = ctx.mesh_upload(c.V, c.T)
        ctx.particles_set(mid, f, b)
        adj = gpu_adjacency(ctx, mid, 6)
        for i in range(6):
            assert adj[i].sum() == 4 and not adj[i, i ^ 1]
    finally:
        ctx.close()


def test_voronoi_after_quench_torus(orc):
    """Gradient-descent quench of 200 particles on the aspect-3 torus on the
    GPU, then the neighbours of the relaxed state on both sides; the net
    defect charge sum (6 - z) vanishes on a torus."""
    from paper_2404_19751_amd import gsim
    m = W.benchmark_torus()
    n = 200
    f, b = W.random_particles(m.nf, n, 101)
    a = np.sqrt(2.0 * W.surface_area(m) / (np.sqrt(3.0) * n))
    sig = 1.2 * a
    ctx = gsim.Context(0, "fp64")
    try:
        mid = ctx.mesh_upload(m.V, m.T)
        ctx.particles_set(mid, f, b)
        ctx.step(mid, gsim.potential("harmonic", 1.0, sig, sig), gsim.integrator("overdamped", 0.05 * sig * sig), 200)
        fq, bq, _, _ = ctx.particles_get(mid)
        g = gpu_adjacency(ctx, mid, n)
    finally:
        ctx.close()
    o = orc.voronoi_neighbours(orc.OracleMesh(m.V, m.T), fq, bq)
    assert np.array_equal(g, o)
    z = g.sum(1)
    assert int(np.sum(6 - z)) == 0
    log(f"[gpu-voronoi] quenched torus: 5-fold {int((z == 5).sum())}, 6-fold {int((z == 6).sum())}, "
        f"7-fold {int((z == 7).sum())}")


def test_voronoi_api_limits():
    """Two-phase capacity protocol, and the error paths: fewer than two
    particles, and more than the bitset holds."""
    import ctypes as C

    from paper_2404_19751_amd import gsim
    m = W.icosphere(3)
    ctx = gsim.Context(0, "fp64")
    try:
        mid = ctx.mesh_upload(m.V, m.T)
        f, b = W.random_particles(m.nf, 50, 103)
        ctx.particles_set(mid, f, b)
        off = np.empty(51, np.int64)
        cnt = C.c_int64(0)
        st = ctx.L.gsim_voronoi_neighbours(ctx.h, mid, off.ctypes.data_as(C.c_void_p), None, 0, C.byref(cnt))
        assert st == gsim.E_CAPACITY and cnt.value > 0
        off2, nbr = ctx.voronoi_neighbours(mid)
        assert off2[-1] == cnt.value == len(nbr)
        ctx.particles_set(mid, f[:1], b[:1])
        with pytest.raises(gsim.GsimError) as e:
            ctx.voronoi_neighbours(mid)
        assert e.value.status == gsim.E_STATE
        f2, b2 = W.random_particles(m.nf, 40000, 105)
        ctx.particles_set(mid, f2, b2)
        with pytest.raises(gsim.GsimError) as e:
            ctx.voronoi_neighbours(mid)
        assert e.value.status == gsim.E_LIMIT
    finally:
        ctx.close()
