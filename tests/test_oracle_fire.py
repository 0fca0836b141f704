"""Pins of the oracle's FIRE minimiser (Bitzek et al., PRL 97, 170201
(2006)) with geodesic Coulomb forces, against values fixed by hand
arithmetic and by known minimum-energy configurations."""
import math

import numpy as np
import pytest

from paper_2404_19751_amd import workloads as W
from tests.util import place


def _xyz(m, face, bary):
    T = m.T[face]
    return np.einsum("ik,ikd->id", bary, m.V[T])


def test_fire_first_two_iterations_by_hand(orc):
    """Two Coulomb particles on a flat sheet, at rest, on a line along x.
    Iteration 1: P = 0 -> velocities reset, dt = dt0/2, v = dt F,
    x += dt^2 F. Iteration 2: P > 0 and v parallel to F, so mixing leaves v
    unchanged; v += dt F', x += dt v. Everything in closed form."""
    m = W.flat_grid(20, 20, 4.0, 4.0)
    om = orc.OracleMesh(m.V, m.T)
    a, b, y = 1.53, 2.41, 2.07
    f, bc = place(m, [np.array([a, y, 0.0]), np.array([b, y, 0.0])])
    pot = dict(kind="coulomb", k=1.0, sigma=1.0, cutoff=math.inf)
    dt0 = 0.2
    ig = dict(kind="fire", dt=dt0)
    st = orc.fire_init(ig)
    v = np.zeros((2, 3))
    f1, b1, v1, st1, info = orc.fire_step(om, f, bc, v, pot, ig, st)
    d = b - a
    dt = dt0 / 2
    assert st1["dt"] == pytest.approx(dt) and st1["alpha"] == pytest.approx(0.1) and st1["n_pos"] == 0
    assert info["P"] == 0.0
    x1 = _xyz(m, f1, b1)
    assert x1[0] == pytest.approx([a - dt * dt / d ** 2, y, 0.0], abs=1e-13)
    assert x1[1] == pytest.approx([b + dt * dt / d ** 2, y, 0.0], abs=1e-13)
    assert v1[0] == pytest.approx([-dt / d ** 2, 0.0, 0.0], abs=1e-13)
    f2, b2, v2, st2, info2 = orc.fire_step(om, f1, b1, v1, pot, ig, st1)
    d1 = d + 2 * dt * dt / d ** 2
    v0 = -dt / d ** 2 - dt / d1 ** 2
    assert info2["P"] > 0 and st2["n_pos"] == 1 and st2["dt"] == pytest.approx(dt)
    x2 = _xyz(m, f2, b2)
    assert x2[0] == pytest.approx([a - dt * dt / d ** 2 + dt * v0, y, 0.0], abs=1e-12)
    assert v2[1] == pytest.approx([-v0, 0.0, 0.0], abs=1e-12)


def test_fire_step_size_adaptation(orc):
    """After more than n_min = 5 consecutive iterations with P > 0 the step
    grows by f_inc = 1.1 per iteration (up to 10 dt0) and alpha shrinks by
    f_alpha = 0.99."""
    m = W.flat_grid(20, 20, 4.0, 4.0)
    om = orc.OracleMesh(m.V, m.T)
    f, bc = place(m, [np.array([1.83, 2.05, 0.0]), np.array([2.27, 2.05, 0.0])])
    pot = dict(kind="coulomb", k=1.0, sigma=1.0, cutoff=math.inf)
    ig = dict(kind="fire", dt=0.01)
    st = orc.fire_init(ig)
    v = np.zeros((2, 3))
    dts, alphas = [], []
    for _ in range(9):
        f, bc, v, st, info = orc.fire_step(om, f, bc, v, pot, ig, st)
        dts.append(st["dt"])
        alphas.append(st["alpha"])
    # iteration 1 resets (dt0/2); iterations 2..6 keep dt; 7, 8, 9 grow it
    assert dts[:6] == pytest.approx([0.005] * 6)
    assert dts[6:] == pytest.approx([0.005 * 1.1, 0.005 * 1.1 ** 2, 0.005 * 1.1 ** 3])
    assert alphas[6:] == pytest.approx([0.1 * 0.99, 0.1 * 0.99 ** 2, 0.1 * 0.99 ** 3])


def _relax(orc, m, n, seed, iters, dt0):
    om = orc.OracleMesh(m.V, m.T)
    f, b = W.random_particles(m.nf, n, seed)
    pot = dict(kind="coulomb", k=1.0, sigma=1.0, cutoff=math.inf)
    ig = dict(kind="fire", dt=dt0, max_disp=0.5 * W.mean_edge_length(m))
    st = orc.fire_init(ig)
    v = np.zeros((n, 3))
    E0 = None
    for _ in range(iters):
        f, b, v, st, info = orc.fire_step(om, f, b, v, pot, ig, st)
        if E0 is None:
            E0 = info["E"]
    pr = orc.geodesic_pairs(om, f, b, math.inf)
    return pr, E0, info["E"], info["F"]


def test_fire_two_particles_go_antipodal(orc):
    """Two charges on the unit icosphere end up (nearly) antipodal: their
    geodesic distance approaches the half circumference pi (slightly less
    on the inscribed polyhedron)."""
    m = W.icosphere(3)
    pr, E0, E1, F = _relax(orc, m, 2, 5, 150, 0.05)
    d = pr.dist[0]
    assert 0.985 * math.pi < d <= math.pi + 1e-9
    assert E1 < E0


def test_fire_thomson_four_is_tetrahedral(orc):
    """Four charges minimise the Coulomb energy at the vertices of a regular
    tetrahedron (the Thomson problem for N = 4): all six geodesic distances
    equal arccos(-1/3) on the unit sphere, up to the polyhedral mesh error.
    (From some starts FIRE stops at the square on a great circle, a saddle
    of the energy; this start reaches the minimum.)"""
    m = W.icosphere(3)
    pr, E0, E1, F = _relax(orc, m, 4, 8, 250, 0.05)
    d = pr.dist.reshape(4, 3)
    target = math.acos(-1.0 / 3.0)
    assert np.abs(d / target - 1.0).max() < 0.02, d
    assert d.std() / d.mean() < 0.005, d
    assert E1 < E0
