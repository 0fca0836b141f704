"""Pins of the oracle's restricted Voronoi neighbours (the in-surface
Voronoi diagram of Sec. 5), against values fixed by symmetry and topology:
regular polyhedra, a triangular lattice, and the Euler characteristic of
the surface (a Voronoi diagram of a closed surface is dual to a
triangulation, so the coordination numbers z_i satisfy
sum_i (6 - z_i) = 6 chi: 12 on a sphere, 0 on a torus)."""
import numpy as np

from paper_2404_19751_amd import workloads as W
from tests.util import place


def test_icosahedron_points_have_five_neighbours(orc):
    """The 12 icosahedron vertices on a subdivided icosphere: every particle
    has exactly its 5 nearest points as neighbours."""
    m = W.icosphere(3)
    om = orc.OracleMesh(m.V, m.T)
    f, b = place(m, m.V[:12])
    adj = orc.voronoi_neighbours(om, f, b)
    assert (adj.sum(1) == 5).all()
    d = np.linalg.norm(m.V[:12, None] - m.V[None, :12], axis=2)
    near = np.abs(d - np.sort(d, axis=1)[:, 1:2]) < 1e-9
    assert np.array_equal(adj, near)


def test_cube_face_centres_are_octahedral(orc):
    """The 6 face centres of a cube: each neighbours the 4 centres of the
    adjacent faces and not the opposite one."""
    m = W.cube(3)
    om = orc.OracleMesh(m.V, m.T)
    c = 0.5 * (m.V.min(0) + m.V.max(0))
    h = 0.5 * (m.V.max(0) - m.V.min(0))
    pts = []
    for ax in range(3):
        for sgn in (1.0, -1.0):
            p = c.copy()
            p[ax] += sgn * h[ax]
            pts.append(p)
    f, b = place(m, pts)
    adj = orc.voronoi_neighbours(om, f, b)
    for i in range(6):
        opp = i ^ 1
        assert adj[i].sum() == 4 and not adj[i, opp]


def test_triangular_lattice_has_six_neighbours(orc):
    """A triangular lattice of spacing a on a flat sheet: every point away
    from the sheet's boundary has exactly the 6 lattice points at distance a
    as neighbours."""
    m = W.flat_grid(24, 24, 6.0, 6.0)
    om = orc.OracleMesh(m.V, m.T)
    a = 0.5
    pts = []
    for j in range(12):
        for i in range(12):
            x = 0.4 + a * i + 0.5 * a * (j % 2)
            y = 0.4 + a * np.sqrt(3.0) / 2.0 * j
            if x < 5.9 and y < 5.9:
                pts.append([x, y, 0.0])
    pts = np.array(pts)
    f, b = place(m, pts)
    adj = orc.voronoi_neighbours(om, f, b)
    inner = (pts[:, 0] > 1.5) & (pts[:, 0] < 4.5) & (pts[:, 1] > 1.5) & (pts[:, 1] < 4.5)
    assert inner.sum() >= 20
    d = np.linalg.norm(pts[:, None] - pts[None], axis=2)
    for i in np.nonzero(inner)[0]:
        assert adj[i].sum() == 6
        assert np.allclose(d[i, adj[i]], a, atol=1e-9)


def test_euler_characteristic_sphere_and_torus(orc):
    """Random particles: sum (6 - z) = 12 on a sphere and 0 on a torus."""
    for m, n, seed, chi in ((W.icosphere(4), 150, 81, 2), (W.benchmark_torus(), 300, 83, 0)):
        om = orc.OracleMesh(m.V, m.T)
        f, b = W.random_particles(m.nf, n, seed)
        adj = orc.voronoi_neighbours(om, f, b)
        assert np.array_equal(adj, adj.T) and not adj.diagonal().any()
        z = adj.sum(1)
        assert int(np.sum(6 - z)) == 6 * chi
        assert z.min() >= 3


def test_two_particles_are_neighbours(orc):
    m = W.icosphere(2)
    om = orc.OracleMesh(m.V, m.T)
    f, b = W.random_particles(m.nf, 2, 85)
    adj = orc.voronoi_neighbours(om, f, b)
    assert adj[0, 1] and adj[1, 0]
