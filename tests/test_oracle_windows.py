"""The window-propagation oracle (Sec. 2.2: the exact continuous-Dijkstra
method with windows trimmed to the pointwise minimum on every edge) pinned
to closed forms, and to the brute-force enumeration oracle on the
workloads: two independent routes to the same exact distances."""
import math

import numpy as np
import pytest

from paper_2404_19751_amd import workloads as W
from tests.util import interior_points, pair_dict, place


def _win(orc, m, f, b, cut, sources=None):
    om = orc.OracleMesh(m.V, m.T)
    return om, orc.geodesic_pairs_windows(om, f, b, cut, sources=sources)


# ---------------------------------------------------------- closed forms ----
def test_flat_grid_is_euclidean(orc):
    g = W.flat_grid(6, 5, 1.2, 1.0)
    f, b = W.random_particles(g.nf, 40, 11)
    om, pr = _win(orc, g, f, b, 0.45)
    x = om.xyz(f, b)
    n_exp = 0
    for i in range(40):
        got = pair_dict(pr, i)
        for j in range(40):
            d = np.linalg.norm(x[j] - x[i])
            if j == i or d >= 0.45:
                assert j not in got
                continue
            n_exp += 1
            p = got[j]
            assert abs(pr.dist[p] - d) <= 1e-13
            assert np.linalg.norm(pr.tan[p] - (x[j] - x[i]) / d) <= 1e-12
    assert n_exp == pr.off[-1] > 50
    assert pr.counters["launches"] > 0  # boundary vertices are pseudo-sources


def test_corrugated_sheet_develops_to_plane(orc):
    """Planar quads: distance = Euclidean distance in the developed plane."""
    m = W.corrugated_sheet(24, 6)
    x = m.meta["x"]
    chord = np.hypot(np.diff(x), np.diff(np.sin(x)))
    S = np.concatenate([[0.0], np.cumsum(chord)])

    def s_of(px):
        i = min(np.searchsorted(x, px, side="right") - 1, len(x) - 2)
        return S[i] + (px - x[i]) / (x[i + 1] - x[i]) * chord[i]

    f, b = interior_points(m, 30, 5)
    om, pr = _win(orc, m, f, b, 1.5)
    P = om.xyz(f, b)
    sy = np.array([[s_of(p[0]), p[1]] for p in P])
    cnt = 0
    for i in range(30):
        got = pair_dict(pr, i)
        for j in range(30):
            d = np.linalg.norm(sy[j] - sy[i])
            if j != i and d < 1.5 - 1e-9:
                cnt += 1
                assert abs(pr.dist[got[j]] - d) < 1e-12
    assert cnt > 40


def test_sources_on_edges(orc):
    """Particles on grid edges of the developed sheet (the source term covers
    both faces of the edge)."""
    m = W.corrugated_sheet(16, 2, sy=1.0)
    xs = [math.pi / 4, 5 * math.pi / 4, 3 * math.pi / 4]
    pts = [(xa, 0.3, math.sin(xa)) for xa in xs]
    f, b = place(m, pts)
    assert all((bb <= 0.0).sum() == 1 for bb in b)
    om, pr = _win(orc, m, f, b, 20.0)
    ref = orc.geodesic_pairs(om, f, b, 20.0)
    assert np.array_equal(pr.nbr, ref.nbr)
    assert np.abs(pr.dist - ref.dist).max() < 1e-12


def test_prism_wraparound(orc):
    n, R = 6, 1.0
    m = W.prism(n, R, 1.0, nz=3)
    side = 2 * R * math.sin(math.pi / n)
    C = n * side

    def pt(s, z):
        k = int(s // side) % n
        t = (s - (s // side) * side) / side
        a = np.array([R * math.cos(2 * math.pi * k / n), R * math.sin(2 * math.pi * k / n)])
        c = np.array([R * math.cos(2 * math.pi * (k + 1) / n), R * math.sin(2 * math.pi * (k + 1) / n)])
        q = (1 - t) * a + t * c
        return (q[0], q[1], z)

    coords = [(0.3, 0.2), (2.9, 0.7), (5.6, 0.5), (1.7, 0.9), (0.3 + C / 2, 0.2)]
    f, b = place(m, [pt(s, z) for s, z in coords])
    _, pr = _win(orc, m, f, b, math.inf)
    for i in range(len(coords)):
        got = pair_dict(pr, i)
        for j in range(len(coords)):
            if j == i:
                continue
            ds, dz = coords[j][0] - coords[i][0], coords[j][1] - coords[i][1]
            d = min(math.hypot(ds + k * C, dz) for k in (-1, 0, 1))
            assert abs(pr.dist[got[j]] - d) < 1e-12


def _cone_point(m, theta, n, r, phi):
    a = theta / n
    k = int(phi // a) % n
    al = phi - k * a
    apex, r1, r2 = m.V[0], m.V[1 + k], m.V[1 + (k + 1) % n]
    e1 = (r1 - apex) / np.linalg.norm(r1 - apex)
    w = r2 - apex
    w = w - np.dot(w, e1) * e1
    e2 = w / np.linalg.norm(w)
    return apex + r * (math.cos(al) * e1 + math.sin(al) * e2)


@pytest.mark.parametrize("theta,n", [(1.5 * np.pi, 6), (2.5 * np.pi, 8), (3.2 * np.pi, 10)])
def test_cone_fan(orc, theta, n):
    """Law of cosines in the opened-up cone below an angular gap of pi, else
    the path bends at the apex (a saddle when theta > 2 pi): d = r1 + r2,
    with the tangent towards the apex."""
    m = W.cone_fan(theta, n)
    rmax = 0.9 * math.cos(theta / (2 * n))
    rng = np.random.default_rng(3)
    pol = [(rmax * (0.15 + 0.8 * rng.random()), theta * rng.random()) for _ in range(14)]
    f, b = place(m, [_cone_point(m, theta, n, r, p) for r, p in pol])
    om, pr = _win(orc, m, f, b, math.inf)
    x = om.xyz(f, b)
    for i, (ri, pi_) in enumerate(pol):
        got = pair_dict(pr, i)
        for j, (rj, pj) in enumerate(pol):
            if j == i:
                continue
            dp = abs(pi_ - pj)
            dp = min(dp, theta - dp)
            d = math.sqrt(ri * ri + rj * rj - 2 * ri * rj * math.cos(dp)) if dp < math.pi else ri + rj
            p = got[j]
            assert abs(pr.dist[p] - d) < 1e-12, (i, j, pr.dist[p], d)
            if dp > math.pi + 1e-6:
                to_apex = (m.V[0] - x[i]) / np.linalg.norm(m.V[0] - x[i])
                assert np.linalg.norm(pr.tan[p] - to_apex) < 1e-9


def test_l_shape_reflex_corner(orc):
    """A boundary pseudo-source: paths that would leave the region bend at
    the reflex corner c."""
    m = W.l_shape(4)
    pts = [(1.8, 0.6, 0), (0.6, 1.8, 0), (1.7, 0.3, 0), (0.3, 1.55, 0), (0.4, 0.4, 0)]
    f, b = place(m, pts)
    _, pr = _win(orc, m, f, b, math.inf)
    c = np.array([1.0, 1.0, 0.0])
    P = np.array(pts, float)
    for i in range(5):
        got = pair_dict(pr, i)
        for j in range(5):
            if j == i:
                continue
            s, t = P[i], P[j]
            u = np.linspace(0, 1, 2001)[:, None]
            seg = s + u * (t - s)
            leaves = np.any((seg[:, 0] > 1 + 1e-9) & (seg[:, 1] > 1 + 1e-9))
            d = (np.linalg.norm(s - c) + np.linalg.norm(c - t)) if leaves else np.linalg.norm(t - s)
            assert abs(pr.dist[got[j]] - d) < 1e-12
            if leaves:
                assert np.linalg.norm(pr.tan[got[j]] - (c - s) / np.linalg.norm(c - s)) < 1e-9


def test_tetrahedron_and_cube(orc):
    m = W.tetrahedron(1.0)
    V = m.V
    pts = [(V[0] + V[1]) / 2, (V[2] + V[3]) / 2, V[[0, 1, 2]].mean(0), V[[1, 2, 3]].mean(0)]
    f, b = place(m, pts)
    _, pr = _win(orc, m, f, b, math.inf)
    assert abs(pr.dist[pair_dict(pr, 0)[1]] - 1.0) < 1e-12
    assert abs(pr.dist[pair_dict(pr, 2)[3]] - 1 / math.sqrt(3)) < 1e-12
    m = W.cube(3)
    f, b = place(m, [(0.2, 0.3, 1), (1, 0.6, 0.1), (0.5, 0.5, 0), (0.5, 0.5, 1)])
    _, pr = _win(orc, m, f, b, math.inf)
    p = pair_dict(pr, 0)[1]
    assert abs(pr.dist[p] - math.sqrt(2.98)) < 1e-12
    t = np.array([1.7, 0.3, 0.0]) / math.hypot(1.7, 0.3)
    assert np.linalg.norm(pr.tan[p] - t) < 1e-12
    assert abs(pr.dist[pair_dict(pr, 3)[2]] - 2.0) < 1e-12


def test_rejects_source_on_vertex(orc):
    m = W.icosphere(2)
    f = np.array([3, 7], np.int32)
    b = np.array([[1.0, 0.0, 0.0], [0.2, 0.3, 0.5]])
    _, pr = _win(orc, m, f, b, 10.0)
    assert pr.counters["rejected"] == 1 and pr.off[1] == 0 and pr.off[2] == 1


# ---------------------------------- agreement with the brute-force oracle ----
CASES = {
    "c1": lambda: (W.workload("c1"), None, None),
    "c2": lambda: (W.workload("c2"), np.arange(0, 1000, 2), None),
    "c4": lambda: (W.workload("c4"), np.arange(0, 20000, 50), None),
    "torus_s1": lambda: (W.workload("torus_nve_2048_1.0"), np.arange(0, 2048, 16), None),
    "ico3_all": lambda: (W.workload("c1"), None, math.inf),
}


@pytest.mark.parametrize("case", list(CASES))
def test_matches_enumeration(orc, case):
    """Same rows, distances within 1e-12 relative, the same tangent where the
    shortest path is unique and a tangent of the tie set where it is not;
    the same pseudo-source vertices reached below the bound."""
    w, src, cut = CASES[case]()
    cut = w.potential["cutoff"] if cut is None else cut
    src = None if src is None else src.astype(np.int32)
    om = orc.OracleMesh(w.mesh.V, w.mesh.T)
    a = orc.geodesic_pairs(om, w.face, w.bary, cut, sources=src)
    b = orc.geodesic_pairs_windows(om, w.face, w.bary, cut, sources=src)
    assert np.array_equal(a.off, b.off) and np.array_equal(a.nbr, b.nbr)
    assert len(a.dist) > 200
    assert np.all(np.abs(b.dist - a.dist) <= 1e-12 * a.dist)
    uniq = (a.flags & 1) == 0
    assert np.linalg.norm(b.tan - a.tan, axis=1)[uniq].max() < 1e-12
    for p in np.nonzero(~uniq)[0]:
        assert np.linalg.norm(a.ties(p) - b.tan[p], axis=1).min() < 1e-12
    assert b.counters["launches"] == a.counters["roots"]
    assert b.counters["rejected"] == a.counters["rejected"] == 0
    # trimming: the exact method propagates fewer windows than enumeration
    assert b.counters["propagated"] < a.counters["windows"]
