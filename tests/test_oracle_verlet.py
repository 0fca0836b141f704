"""Pins of the oracle's velocity-Verlet (leapfrog) integrator on curved
surfaces: exact time reversibility (a property of the scheme that a wrong
kick, drift order, transport or force sign breaks) and energy conservation."""
import numpy as np

from paper_2404_19751_amd import workloads as W


def _energy(orc, om, f, b, v_half, pot, dt):
    """Total energy at integer time: v_k = v_{k-1/2} + (dt/2) F(x_k)."""
    pr = orc.geodesic_pairs(om, f, b, pot["cutoff"])
    F, U = orc.forces(len(f), pr, pot["kind"], pot["k"], pot["sigma"])
    v = v_half + 0.5 * dt * F
    return 0.5 * float(np.sum(v * v)) + U, F


def test_verlet_time_reversible_on_sphere(orc):
    """Forward K steps, then the same scheme started from the reversed
    velocity -(v_{K-1/2} + dt F_K) walks every particle back to its start."""
    m = W.icosphere(3)
    om = orc.OracleMesh(m.V, m.T)
    n = 8
    f0, b0 = W.random_particles(m.nf, n, 61)
    pot = dict(kind="harmonic", k=1.0, sigma=0.9, cutoff=0.9)
    ig = dict(kind="verlet", dt=0.02)
    rng = np.random.default_rng(3)
    # initial tangent velocities in each particle's face plane
    v = rng.normal(size=(n, 3)) * 0.5
    nrm = np.cross(m.V[m.T[f0, 1]] - m.V[m.T[f0, 0]], m.V[m.T[f0, 2]] - m.V[m.T[f0, 0]])
    nrm /= np.linalg.norm(nrm, axis=1)[:, None]
    v -= np.sum(v * nrm, axis=1)[:, None] * nrm
    f, b = f0.copy(), b0.copy()
    flags = np.zeros(n, np.int64)
    K = 40
    crossings = 0
    for _ in range(K):
        f, b, v, info = orc.verlet_step(om, f, b, v, pot, ig)
        flags |= info["walk_flags"]
        crossings += info["walk"]["crossings"]
    assert crossings > 20
    _, FK = _energy(orc, om, f, b, v, pot, ig["dt"])
    w = -(v + ig["dt"] * FK)
    for _ in range(K):
        f, b, w, info = orc.verlet_step(om, f, b, w, pot, ig)
        flags |= info["walk_flags"]
    ok = flags & 3 == 0
    assert ok.all()
    assert np.array_equal(f, f0)
    assert np.abs(b - b0).max() < 1e-9


def test_verlet_energy_conserved(orc):
    """Harmonic repulsion on a flat sheet (no boundary reached): the total
    energy at integer times stays within O(dt^2) of its start, with no drift."""
    m = W.flat_grid(30, 30, 6.0, 6.0)
    om = orc.OracleMesh(m.V, m.T)
    n = 12
    f, b = W.random_particles(m.nf, n, 67)
    # keep everyone near the middle
    xyz = np.einsum("ik,ikd->id", b, m.V[m.T[f]])
    sel = np.linalg.norm(xyz[:, :2] - 3.0, axis=1) < 2.5
    f, b = f[sel], b[sel]
    n = len(f)
    pot = dict(kind="harmonic", k=1.0, sigma=1.2, cutoff=1.2)
    dt = 0.01
    ig = dict(kind="verlet", dt=dt)
    v = np.zeros((n, 3))
    E0, _ = _energy(orc, om, f, b, v, pot, dt)
    Es = []
    for k in range(300):
        f, b, v, info = orc.verlet_step(om, f, b, v, pot, ig)
        if k % 10 == 9:
            Es.append(_energy(orc, om, f, b, v, pot, dt)[0])
    Es = np.array(Es)
    assert E0 > 0.05
    assert np.abs(Es - E0).max() < 2e-3 * E0
    assert abs(np.mean(Es[-5:]) - np.mean(Es[:5])) < 1e-3 * E0
