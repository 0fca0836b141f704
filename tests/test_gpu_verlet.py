"""GPU tests of velocity Verlet (leapfrog form, NVE) with parallel-transported
velocities: trajectory parity with the oracle, exact time reversal on a
curved surface, and energy conservation on the benchmark torus."""
import sys

import numpy as np
import pytest

from paper_2404_19751_amd import workloads as W

pytestmark = pytest.mark.gpu


def log(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _setup(m, n, seed, speed):
    f, b = W.random_particles(m.nf, n, seed)
    rng = np.random.default_rng(seed)
    v = rng.normal(size=(n, 3)) * speed
    nrm = np.cross(m.V[m.T[f, 1]] - m.V[m.T[f, 0]], m.V[m.T[f, 2]] - m.V[m.T[f, 0]])
    nrm /= np.linalg.norm(nrm, axis=1)[:, None]
    v -= np.sum(v * nrm, axis=1)[:, None] * nrm
    return f, b, v


def test_verlet_trajectory_matches_oracle(orc):
    """Ten Verlet steps on the GPU (FP64) against ten oracle steps from the
    same state, compared after every step."""
    from paper_2404_19751_amd import gsim
    m = W.icosphere(3)
    om = orc.OracleMesh(m.V, m.T)
    f, b, v = _setup(m, 20, 71, 0.5)
    pot_o = dict(kind="harmonic", k=1.0, sigma=0.9, cutoff=0.9)
    ig_o = dict(kind="verlet", dt=0.02)
    ctx = gsim.Context(0, "fp64")
    try:
        mid = ctx.mesh_upload(m.V, m.T)
        ctx.particles_set(mid, f, b, v)
        pot = gsim.potential("harmonic", 1.0, 0.9, 0.9)
        ig = gsim.integrator("verlet", 0.02)
        flags = np.zeros(20, np.int64)
        for k in range(10):
            ctx.step(mid, pot, ig, 1)
            f, b, v, info = orc.verlet_step(om, f, b, v, pot_o, ig_o)
            flags |= info["walk_flags"]
            fg, bg, vg, _ = ctx.particles_get(mid)
            ok = flags & 3 == 0
            assert np.array_equal(fg[ok], f[ok]), f"step {k}"
            assert np.abs(bg[ok] - b[ok]).max() < 1e-10, f"step {k}"
            assert np.abs(vg[ok] - v[ok]).max() < 1e-10, f"step {k}"
        log("[gpu-verlet] 10 steps match the oracle")
    finally:
        ctx.close()


def test_verlet_time_reversal():
    """Forward 60 steps (graph replays), then from the reversed velocity
    -(v_{K-1/2} + dt F_K) 60 more: every particle returns to its start."""
    from paper_2404_19751_amd import gsim
    m = W.torus(1.0, 0.3, 40, 16)
    n = 60
    f0, b0, v0 = _setup(m, n, 73, 0.4)
    dt = 0.01
    ctx = gsim.Context(0, "fp64")
    try:
        mid = ctx.mesh_upload(m.V, m.T)
        ctx.particles_set(mid, f0, b0, v0)
        pot = gsim.potential("harmonic", 1.0, 0.3, 0.3)
        ig = gsim.integrator("verlet", dt)
        ctx.step(mid, pot, ig, 60)
        f, b, v, _ = ctx.particles_get(mid)
        F, _ = ctx.compute_forces(mid, pot)
        ctx.particles_set(mid, f, b, -(v + dt * F))
        ctx.step(mid, pot, ig, 60)
        f1, b1, _, _ = ctx.particles_get(mid)
        assert np.array_equal(f1, f0)
        err = np.abs(b1 - b0).max()
        log(f"[gpu-verlet] time reversal: max barycentric error {err:.2e}")
        assert err < 1e-8
    finally:
        ctx.close()


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_verlet_energy_on_benchmark_torus(prec):
    """NVE on the benchmark torus: total energy at integer times (kinetic
    from v_k = v_{k-1/2} + (dt/2) F_k) stays close to its start."""
    from paper_2404_19751_amd import gsim
    w = W.workload("torus_nve_2048_0.5")
    dt = 0.002
    ctx = gsim.Context(0, prec)
    try:
        mid = ctx.mesh_upload(w.mesh.V, w.mesh.T)
        ctx.particles_set(mid, w.face, w.bary)
        pot = gsim.potential("harmonic", 1.0, 0.5, 0.5)
        ig = gsim.integrator("verlet", dt)

        def energy():
            F, U = ctx.compute_forces(mid, pot)
            _, _, v, _ = ctx.particles_get(mid)
            vk = v + 0.5 * dt * F
            return 0.5 * float(np.sum(vk * vk)) + U, U

        E0, U0 = energy()
        Es = []
        for _ in range(10):
            ctx.step(mid, pot, ig, 20)
            Es.append(energy()[0])
        Es = np.array(Es)
        rel = np.abs(Es - E0).max() / E0
        log(f"[gpu-verlet] {prec}: E0={E0:.6f} (U0={U0:.6f}) max rel drift {rel:.2e}")
        assert rel < 5e-3
    finally:
        ctx.close()
