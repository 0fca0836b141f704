"""Pins for the oracle's shift walk, force sum, integrators and RNG."""
import math
import os

import numpy as np
import pytest

from paper_2404_19751_amd import workloads as W
from tests.util import locate, pair_dict, place

GOLD = os.path.join(os.path.dirname(__file__), "golden")


# ------------------------------------------------------------ RNG pins ----
def test_philox_known_answers(orc):
    for line in open(os.path.join(GOLD, "philox4x32_10_kat.txt")):
        if line.startswith("#") or not line.strip():
            continue
        v = [int(x, 16) for x in line.split()]
        assert orc.philox4x32_10(v[0:4], v[4:6]) == v[6:10]


def test_splitmix64_reference_outputs():
    ref = [int(x, 16) for x in open(os.path.join(GOLD, "splitmix64.txt")) if not x.startswith("#")]
    assert [int(x) for x in W.splitmix64(0, 3)] == ref


def test_box_muller_moments(orc):
    z = np.array([orc.gaussian_pair(7, s, p) for s in range(40) for p in range(100)]).reshape(-1)
    assert abs(z.mean()) < 0.05 and abs(z.var() - 1.0) < 0.06
    a = np.array([orc.gaussian_pair(7, 3, p) for p in range(2000)])
    assert abs(np.corrcoef(a[:, 0], a[:, 1])[0, 1]) < 0.08


# ---------------------------------------------------------- walk (CF2/3) ----
def test_walk_flat_is_vector_addition(orc):
    """In flat space the shift is plain vector addition (Sec. 3.2)."""
    g = W.flat_grid(10, 10, 2.0, 2.0)
    om = orc.OracleMesh(g.V, g.T)
    rng = np.random.default_rng(1)
    x0 = 0.5 + rng.random((60, 2))
    D = (rng.random((60, 2)) - 0.5) * 0.9
    f, b = place(g, [(p[0], p[1], 0.0) for p in x0])
    D3 = np.concatenate([D, 0.3 * np.ones((60, 1))], 1)  # normal part must be removed
    f2, b2, _, st, _ = orc.walk(om, f, b, D3)
    x1 = om.xyz(f2, b2)
    assert np.max(np.abs(x1[:, :2] - (x0 + D))) < 1e-13 and np.all(x1[:, 2] == 0)
    assert st["crossings"] > 20
    for k in range(60):  # the reported face really contains the point
        assert locate(g, x1[k], 1e-12)[0] >= 0 and b2[k].min() >= -1e-15


def test_walk_corrugated_is_developed_addition(orc):
    m = W.corrugated_sheet(24, 6)
    om = orc.OracleMesh(m.V, m.T)
    x = m.meta["x"]
    chord = np.hypot(np.diff(x), np.diff(np.sin(x)))
    S = np.concatenate([[0.0], np.cumsum(chord)])

    def s_of(px):
        i = min(np.searchsorted(x, px, side="right") - 1, len(x) - 2)
        return S[i] + (px - x[i]) / (x[i + 1] - x[i]) * chord[i]

    i0 = np.searchsorted(x, 1.0, side="right") - 1
    z0 = math.sin(x[i0]) + (1.0 - x[i0]) / (x[i0 + 1] - x[i0]) * (math.sin(x[i0 + 1]) - math.sin(x[i0]))
    f, b = place(m, [(1.0, 0.8, z0)])  # a point on the chord surface
    p0 = om.xyz(f, b)[0]
    # direction in the start face: along its developed axes (s, y)
    es = np.array([x[i0 + 1] - x[i0], 0, math.sin(x[i0 + 1]) - math.sin(x[i0])])
    es /= np.linalg.norm(es)
    ds, dy = 3.1, 0.7
    f2, b2, _, st, _ = orc.walk(om, f, b, (ds * es + dy * np.array([0, 1, 0]))[None, :])
    p1 = om.xyz(f2, b2)[0]
    assert abs(s_of(p1[0]) - (s_of(p0[0]) + ds)) < 1e-12 and abs(p1[1] - (p0[1] + dy)) < 1e-12
    assert st["crossings"] >= 8


# ------------------------------------------------------ walk closed loops ----
def test_walk_cube_belt_returns(orc):
    """A straight walk of length 4 around the belt of a unit cube returns to
    the start, in the same face, with the same velocity."""
    m = W.cube(2)
    om = orc.OracleMesh(m.V, m.T)
    f, b = place(m, [(0.3, 0.0, 0.4)])
    v = np.array([[0.0, 0.0, 1.0]])
    f2, b2, v2, st, _ = orc.walk(om, f, b, np.array([[4.0, 0, 0]]), v)
    assert f2[0] == f[0] and np.max(np.abs(b2 - b)) < 1e-13
    assert np.max(np.abs(v2 - v)) < 1e-13 and st["crossings"] >= 8


def test_walk_prism_circumference(orc):
    n, R = 7, 1.0
    m = W.prism(n, R, 1.0, 2)
    om = orc.OracleMesh(m.V, m.T)
    C = 2 * n * R * math.sin(math.pi / n)
    a, c = m.V[0], m.V[1]
    p = 0.35 * a + 0.65 * c + np.array([0, 0, 0.3])
    f, b = place(m, [p])
    t = (c - a) / np.linalg.norm(c - a)
    f2, b2, _, _, _ = orc.walk(om, f, b, (C * t)[None, :])
    assert f2[0] == f[0] and np.max(np.abs(b2 - b)) < 1e-12


def test_holonomy_cube_corner(orc):
    """Parallel transport around a closed loop enclosing one cube corner
    rotates a vector by the angle defect 2 pi - 3 pi/2 = pi/2 (discrete
    Gauss-Bonnet), the transport the shift carries (Sec. 3.2)."""
    m = W.cube(1)
    om = orc.OracleMesh(m.V, m.T)
    A, B, Cc = np.array([0.6, 0.8, 1.0]), np.array([1.0, 0.6, 0.8]), np.array([0.8, 1.0, 0.6])
    legs = [np.array([0.6, -0.2, 0.0]), np.array([0.0, 0.6, -0.2]), np.array([-0.2, 0.0, 0.6])]
    targets = [B, Cc, A]
    f, b = place(m, [A])
    v0 = np.array([[1.0, 0.0, 0.0]])
    v = v0.copy()
    for D, T in zip(legs, targets):
        f, b, v, st, _ = orc.walk(om, f, b, D[None, :], v)
        assert np.linalg.norm(om.xyz(f, b)[0] - T) < 1e-13
        assert st["crossings"] >= 1  # diagonals of the split squares count too
    ang = math.atan2(np.cross(v0[0], v[0]) @ np.array([0, 0, 1.0]), v0[0] @ v[0])
    assert abs(abs(ang) - math.pi / 2) < 1e-12


def test_walk_reversible_and_length(orc):
    m = W.bumpy_sphere(3, 0.12)
    om = orc.OracleMesh(m.V, m.T)
    f, b = W.random_particles(m.nf, 200, 21)
    rng = np.random.default_rng(5)
    D = rng.normal(size=(200, 3)) * 0.25
    f1, b1, vt, st, fl = orc.walk(om, f, b, D, D.copy())
    assert st["crossings"] > 200
    ok = fl == 0
    f2, b2, _, _, _ = orc.walk(om, f1, b1, -vt)
    assert np.array_equal(f2[ok], f[ok]) and np.max(np.abs(b2[ok] - b[ok])) < 1e-11
    # the transported displacement keeps its length and stays in the new face's plane
    Dn = D - (D * om.normal[f]).sum(1, keepdims=True) * om.normal[f]
    assert np.max(np.abs(np.linalg.norm(vt, axis=1) - np.linalg.norm(Dn, axis=1))) < 1e-12
    assert np.max(np.abs((vt * om.normal[f1]).sum(1))) < 1e-12
    assert b1.min() >= -1e-14 and np.max(np.abs(b1.sum(1) - 1)) < 1e-12


def test_walk_vertex_hit_straightest(orc):
    """Walking straight at a vertex of a cone: the path leaves so that the
    angles on both sides are equal (half the angle sum each)."""
    theta, n = 1.5 * np.pi, 6
    m = W.cone_fan(theta, n)
    om = orc.OracleMesh(m.V, m.T)
    apex, r1, r2 = m.V[0], m.V[1], m.V[2]
    e1 = (r1 - apex) / np.linalg.norm(r1 - apex)
    start = apex + 0.5 * e1 + 0.1 * ((r2 - apex) - np.dot(r2 - apex, e1) * e1) / np.linalg.norm(
        (r2 - apex) - np.dot(r2 - apex, e1) * e1)
    f, b = place(m, [start])
    dirv = apex - start
    Lin = np.linalg.norm(dirv)
    f2, b2, _, st, fl = orc.walk(om, f, b, (dirv / Lin * (Lin + 0.3))[None, :])
    assert st["vertex_hits"] == 1
    end = om.xyz(f2, b2)[0]
    assert abs(np.linalg.norm(end - apex) - 0.3) < 1e-12
    # intrinsic polar angle of start and end around the apex differ by theta/2
    def polar(p):
        best = None
        for k in range(n):
            a, c = m.V[1 + k], m.V[1 + (k + 1) % n]
            ea = (a - apex) / np.linalg.norm(a - apex)
            w = p - apex
            ang = math.atan2(np.linalg.norm(np.cross(ea, w)), ea @ w)
            nrm = np.cross(a - apex, c - apex)
            if abs(w @ nrm) < 1e-12 and ang <= theta / n + 1e-12 and np.cross(ea, w) @ nrm >= -1e-12:
                best = k * theta / n + ang
        return best
    d = abs(polar(end) - polar(start))
    assert abs(min(d, theta - d) - theta / 2) < 1e-9


# ------------------------------------------------------------- forces ----
def test_two_body_harmonic(orc):
    """|F| = (k/sigma)(1 - d/sigma), pointing from j away from i's side
    (repulsion; the sign reading of the force sum)."""
    g = W.flat_grid(4, 4)
    om = orc.OracleMesh(g.V, g.T)
    f, b = place(g, [(0.4, 0.45, 0), (0.62, 0.5, 0)])
    pr = orc.geodesic_pairs(om, f, b, 0.5)
    F, E = orc.forces(2, pr, "harmonic", k=2.0, sigma=0.5)
    d = math.hypot(0.22, 0.05)
    u = np.array([0.22, 0.05, 0]) / d
    assert np.allclose(F[0], -(2.0 / 0.5) * (1 - d / 0.5) * u, atol=1e-14)
    assert np.allclose(F[1], -F[0], atol=1e-14)
    assert abs(E - 0.5 * 2.0 * (1 - d / 0.5) ** 2) < 1e-15
    _, Ec = orc.forces(2, orc.geodesic_pairs(om, f, b, 5.0), "coulomb")
    assert abs(Ec - 1 / d) < 1e-13


def test_flat_forces_sum_to_zero(orc):
    g = W.flat_grid(8, 8)
    om = orc.OracleMesh(g.V, g.T)
    f, b = W.random_particles(g.nf, 80, 4)
    pr = orc.geodesic_pairs(om, f, b, 0.3)
    for kind in ("harmonic", "gaussian"):
        F, _ = orc.forces(80, pr, kind, 1.0, 0.3)
        assert np.abs(F.sum(0)).max() < 1e-13 and np.abs(F).max() > 0.1


def test_energy_gradient_finite_difference(orc):
    """F_i . u = -dE/ds along a geodesic shift of particle i (central
    difference): pins the sign convention and the tangents together."""
    m = W.bumpy_sphere(3, 0.1)
    om = orc.OracleMesh(m.V, m.T)
    f, b = W.random_particles(m.nf, 60, 2)
    cut = 0.6
    pr = orc.geodesic_pairs(om, f, b, cut)
    F, _ = orc.forces(60, pr, "gaussian", 1.0, 0.25)  # smooth: no kink at the cutoff
    # the Gaussian has range ~ 0.6 here; pairs beyond the cutoff contribute < 3e-3 -> use large cutoff
    pr = orc.geodesic_pairs(om, f, b, 1.9)
    F, _ = orc.forces(60, pr, "gaussian", 1.0, 0.25)
    eps = 1e-6
    checked = 0
    for i in (0, 7, 19, 33):
        for u in (om.ex[f[i]], om.ey[f[i]]):
            Es = []
            for sgn in (1, -1):
                D = np.zeros((60, 3))
                D[i] = sgn * eps * u
                f2, b2, _, _, _ = orc.walk(om, f, b, D)
                _, E = orc.forces(60, orc.geodesic_pairs(om, f2, b2, 1.9), "gaussian", 1.0, 0.25)
                Es.append(E)
            fd = -(Es[0] - Es[1]) / (2 * eps)
            assert abs(F[i] @ u - fd) < 1e-6 * max(1.0, abs(fd)), (i, F[i] @ u, fd)
            checked += 1
    assert checked == 8


def test_overdamped_and_brownian_displacement(orc):
    m = W.icosphere(2)
    om = orc.OracleMesh(m.V, m.T)
    f = np.arange(10, dtype=np.int32)
    F = np.random.default_rng(0).normal(size=(10, 3))
    D = orc.displacement(om, f, F, dict(kind="overdamped", dt=0.01, mobility=2.0))
    assert np.allclose(D, 0.02 * F, rtol=0, atol=0)
    ig = dict(kind="brownian", dt=0.005, kT=0.1, friction=1.0, seed=3)
    D0 = orc.displacement(om, f, np.zeros((10, 3)), ig, step=5)
    assert np.max(np.abs((D0 * om.normal[f]).sum(1))) < 1e-15  # tangent noise
    ig2 = dict(ig, friction=2.0)
    D2 = orc.displacement(om, f, np.zeros((10, 3)), ig2, step=5)
    assert np.allclose(D2, D0 / math.sqrt(2.0), atol=1e-15)  # amplitude sqrt(2 kT dt / lambda)


def test_force_error_scale_is_first_order_bound():
    """The force-error scale used by the GPU comparisons, |U'| + d |U''|,
    against central differences of the oracle's U' (away from the harmonic
    cutoff's kink), for the three potentials."""
    import oracle as orc
    from tests.util import force_scale
    d = np.linspace(0.05, 0.95, 37)
    for kind in ("harmonic", "coulomb", "gaussian"):
        h = 1e-6 * d
        _, up = orc.potential(kind, d + h, 1.3, 1.0)
        _, um = orc.potential(kind, d - h, 1.3, 1.0)
        _, u0 = orc.potential(kind, d, 1.3, 1.0)
        want = np.abs(u0) + d * np.abs((up - um) / (2 * h))
        assert np.allclose(force_scale(kind, d, 1.3, 1.0), want, rtol=1e-6), kind
