"""Pins for the oracle's open-boundary walk rule and its Brownian noise
amplitude, each against a closed form.

Boundary (the paper treats closed surfaces only; reading A-8: specular
reflection in the face plane at a boundary edge, reversal at a boundary
vertex). On a flat rectangle the reflected walk is a billiard, whose end
point is the unreflected end point folded back into the rectangle (the
method of images), with each velocity component's sign flipped once per
reflection off the walls across it. On the corrugated sheet z = sin x,
which is developable (Sec. 2.1, Eq. (9) example), the same holds in the
developed coordinates (s, y). A walk straight into a convex corner comes
back along its own line.

Noise (Sec. 2.1, the discrete overdamped Langevin update Eq. (2), reading
A-9): with no force, D = sqrt(2 kT dt / lambda) (eta1 e_x + eta2 e_y) with
independent unit normals, so E|D|^2 = 2 (2 kT dt / lambda), each tangent
axis carries 2 kT dt / lambda, the axes are uncorrelated and the mean is 0.
The sample statistics over 2 x 10^4 particle-steps are checked within four
standard errors, which a dropped factor 2, kT or 1/lambda exceeds many
times over."""
import math

import numpy as np

from paper_2404_19751_amd import workloads as W
from tests.util import place


def fold(x, a):
    """Image of coordinate x in [0, a] after reflections off 0 and a, and
    the number of reflections."""
    k = np.floor(x / a).astype(np.int64)
    r = x - k * a
    return np.where(k % 2 == 0, r, a - r), k


def test_walk_reflects_in_flat_rectangle(orc):
    """Random walks in [0,2]x[0,1.5], many of them bouncing several times:
    end point and velocity are the billiard's closed form."""
    sx, sy = 2.0, 1.5
    g = W.flat_grid(8, 6, sx, sy)
    om = orc.OracleMesh(g.V, g.T)
    rng = np.random.default_rng(11)
    n = 200
    x0 = np.stack([0.05 + 1.9 * rng.random(n), 0.05 + 1.4 * rng.random(n)], 1)
    ang = 2 * np.pi * rng.random(n)
    L = 0.3 + 5.0 * rng.random(n)
    D = np.stack([L * np.cos(ang), L * np.sin(ang), np.zeros(n)], 1)
    v = np.stack([np.cos(ang + 0.4), np.sin(ang + 0.4), np.zeros(n)], 1)
    f, b = place(g, [(p[0], p[1], 0.0) for p in x0])
    f2, b2, v2, st, fl = orc.walk(om, f, b, D, v)
    ok = (fl & 3) == 0  # no vertex hit or near-vertex pass
    assert ok.mean() > 0.9 and st["boundary_hits"] > 300
    X, kx = fold(x0[:, 0] + D[:, 0], sx)
    Y, ky = fold(x0[:, 1] + D[:, 1], sy)
    x1 = om.xyz(f2, b2)
    assert np.max(np.abs(x1[ok, 0] - X[ok])) < 1e-12
    assert np.max(np.abs(x1[ok, 1] - Y[ok])) < 1e-12
    assert np.all(x1[:, 2] == 0.0)
    vx = np.where(kx % 2 == 0, 1.0, -1.0) * v[:, 0]
    vy = np.where(ky % 2 == 0, 1.0, -1.0) * v[:, 1]
    assert np.max(np.abs(v2[ok, 0] - vx[ok])) < 1e-12 and np.max(np.abs(v2[ok, 1] - vy[ok])) < 1e-12
    # the number of boundary hits is the number of fold reflections
    _, _, _, st_ok, _ = orc.walk(om, f[ok], b[ok], D[ok], v[ok])
    assert st_ok["boundary_hits"] == int((np.abs(kx) + np.abs(ky))[ok].sum())


def test_walk_single_reflection_mirror_image():
    """One reflection off the wall x = 1: the end point is the mirror image of
    the unreflected end, and the velocity's normal component flips."""
    import oracle as orc
    g = W.flat_grid(5, 5)
    om = orc.OracleMesh(g.V, g.T)
    f, b = place(g, [(0.3, 0.47, 0.0)])
    D = np.array([[1.0, 0.2, 0.0]])
    v = np.array([[0.8, -0.3, 0.0]])
    f2, b2, v2, st, fl = orc.walk(om, f, b, D, v)
    p = om.xyz(f2, b2)[0]
    assert st["boundary_hits"] == 1 and fl[0] == 8
    assert np.max(np.abs(p - np.array([2.0 - 1.3, 0.67, 0.0]))) < 1e-14
    assert np.max(np.abs(v2[0] - np.array([-0.8, -0.3, 0.0]))) < 1e-15


def test_walk_reverses_at_convex_corner(orc):
    """Straight into the corner (0, 0) of the square (a boundary vertex): the
    walk comes back along its own line for the rest of its length, the
    velocity reversed."""
    g = W.flat_grid(4, 4)
    om = orc.OracleMesh(g.V, g.T)
    for start, rest in (((0.3, 0.1), 0.17), ((0.05, 0.21), 0.4)):
        s = np.array([start[0], start[1], 0.0])
        u = -s / np.linalg.norm(s)
        L = np.linalg.norm(s) + rest
        f, b = place(g, [s])
        v = np.array([[0.0, 0.0, 0.0]]) + 2.5 * u
        f2, b2, v2, st, fl = orc.walk(om, f, b, (L * u)[None, :], v)
        p = om.xyz(f2, b2)[0]
        assert st["vertex_hits"] == 1 and (fl[0] & 1)
        assert np.linalg.norm(p - rest * (-u)) < 1e-13, (p, rest * (-u))
        assert np.linalg.norm(v2[0] + 2.5 * u) < 1e-13
    # the opposite corner (4/4, 4/4) of a coarser grid, from inside
    c = np.array([1.0, 1.0, 0.0])
    s = np.array([0.62, 0.91, 0.0])
    u = (c - s) / np.linalg.norm(c - s)
    f, b = place(g, [s])
    f2, b2, _, st, _ = orc.walk(om, f, b, ((np.linalg.norm(c - s) + 0.25) * u)[None, :])
    assert st["vertex_hits"] == 1
    assert np.linalg.norm(om.xyz(f2, b2)[0] - (c - 0.25 * u)) < 1e-13


def test_walk_reflects_on_developed_corrugated_sheet(orc):
    """On the developable sheet z = sin x, x in [0, 2 pi], y in [0, 2], the
    reflected walk is the billiard in the developed rectangle
    [0, S] x [0, 2] (S the total chord length)."""
    m = W.corrugated_sheet(24, 6)
    om = orc.OracleMesh(m.V, m.T)
    x = m.meta["x"]
    chord = np.hypot(np.diff(x), np.diff(np.sin(x)))
    S = np.concatenate([[0.0], np.cumsum(chord)])
    Stot = S[-1]

    def s_of(px):
        i = min(np.searchsorted(x, px, side="right") - 1, len(x) - 2)
        return S[i] + (px - x[i]) / (x[i + 1] - x[i]) * chord[i]

    def point_at(s, y):
        i = min(np.searchsorted(S, s, side="right") - 1, len(x) - 2)
        t = (s - S[i]) / chord[i]
        px = x[i] + t * (x[i + 1] - x[i])
        pz = math.sin(x[i]) + t * (math.sin(x[i + 1]) - math.sin(x[i]))
        return np.array([px, y, pz]), i

    checked = 0
    for s0, y0, ds, dy in ((1.3, 0.7, -3.0, 0.45), (5.0, 1.2, 4.4, -3.1), (2.2, 0.3, 9.0, 5.5)):
        p0, i0 = point_at(s0, y0)
        f, b = place(m, [p0])
        es = np.array([x[i0 + 1] - x[i0], 0.0, math.sin(x[i0 + 1]) - math.sin(x[i0])])
        es /= np.linalg.norm(es)
        f2, b2, _, st, fl = orc.walk(om, f, b, (ds * es + dy * np.array([0.0, 1.0, 0.0]))[None, :])
        if fl[0] & 3:
            continue
        p1 = om.xyz(f2, b2)[0]
        Sx, _ = fold(np.array([s0 + ds]), Stot)
        Yy, _ = fold(np.array([y0 + dy]), 2.0)
        assert st["boundary_hits"] >= 1
        assert abs(s_of(p1[0]) - Sx[0]) < 1e-11 and abs(p1[1] - Yy[0]) < 1e-12
        checked += 1
    assert checked == 3


def noise_moments(orc, om, f, ig, steps):
    """Displacements with zero force over `steps` steps: their components
    along each particle's face axes."""
    ex, ey = om.ex[f], om.ey[f]
    a, c = [], []
    for s in range(steps):
        D = orc.displacement(om, f, np.zeros((len(f), 3)), ig, step=s)
        a.append((D * ex).sum(1))
        c.append((D * ey).sum(1))
    return np.concatenate(a), np.concatenate(c)


def test_brownian_amplitude_closed_form(orc):
    m = W.icosphere(3)
    om = orc.OracleMesh(m.V, m.T)
    n, steps = 500, 40
    f = (np.arange(n) * 7 % m.nf).astype(np.int32)
    N = n * steps
    for kT, lam, dt in ((0.1, 1.0, 0.005), (0.3, 2.0, 0.01), (2.0, 0.5, 1e-3)):
        ig = dict(kind="brownian", dt=dt, kT=kT, friction=lam, seed=9)
        s2 = 2.0 * kT * dt / lam  # variance per tangent axis
        a, c = noise_moments(orc, om, f, ig, steps)
        msd = float(np.mean(a * a + c * c))
        # |D|^2 / s2 is chi-square with 2 degrees of freedom: mean 2, variance 4
        assert abs(msd / (2.0 * s2) - 1.0) <= 4.0 / math.sqrt(N), (kT, lam, dt, msd, 2 * s2)
        # each axis: chi-square(1) / s2, variance 2
        for comp in (a, c):
            assert abs(float(np.mean(comp * comp)) / s2 - 1.0) <= 4.0 * math.sqrt(2.0 / N)
            assert abs(float(np.mean(comp))) <= 4.0 * math.sqrt(s2 / N)
        assert abs(float(np.mean(a * c))) <= 4.0 * s2 / math.sqrt(N)


def test_brownian_drift_term(orc):
    """With kT = 0 the update is the deterministic drift D = (dt / lambda) F."""
    m = W.icosphere(2)
    om = orc.OracleMesh(m.V, m.T)
    f = np.arange(12, dtype=np.int32)
    F = np.random.default_rng(3).normal(size=(12, 3))
    D = orc.displacement(om, f, F, dict(kind="brownian", dt=0.02, kT=0.0, friction=4.0, seed=1), step=3)
    assert np.array_equal(D, (0.02 / 4.0) * F)
