"""GPU parity on the open height-field workload at full size: 199,712 faces
with an open boundary, N = 20,000, harmonic sigma = cutoff = 3 mean edge
lengths, Brownian dynamics (kT 0.1, friction 1, dt 0.005).

Every source is compared with the CPU oracle (neighbour sets bit-exact,
distances and tangents within 1e-12 in FP64 mode and 1e-5 in FP32-mixed
mode). The step is checked as stage parity: the GPU and the oracle start
from the same FP64 state, and their faces must agree bit for bit."""
import sys

import numpy as np
import pytest

from paper_2404_19751_amd import workloads as W
from tests.test_gpu_fp32 import compare32
from tests.test_gpu_parity import compare_pairs
from tests.util import oracle_band, step_within_force_bound

pytestmark = pytest.mark.gpu


def log(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def c4(orc):
    w = W.workload("c4")
    om = orc.OracleMesh(w.mesh.V, w.mesh.T)
    log(f"[gpu-c4] oracle pairs: nf={w.mesh.nf} n={len(w.face)} cutoff={w.potential['cutoff']:.5f}")
    o = orc.geodesic_pairs(om, w.face, w.bary, w.potential["cutoff"])
    o32 = orc.geodesic_pairs(om, w.face, w.bary, w.potential["cutoff"], **oracle_band("fp32"))
    log(f"[gpu-c4] oracle pairs done: {len(o.dist)} pairs")
    return w, om, o, o32


def _ctx(prec):
    from paper_2404_19751_amd import gsim
    return gsim.Context(0, prec)


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_c4_pairs_full(c4, prec):
    w, om, o, o32 = c4
    ctx = _ctx(prec)
    try:
        mid = ctx.mesh_upload(w.mesh.V, w.mesh.T)
        info = ctx.mesh_info(mid)
        assert info["n_boundary_edges"] == 4 * 316
        ctx.particles_set(mid, w.face, w.bary)
        log(f"[gpu-c4] {prec} geodesic_pairs")
        g = ctx.geodesic_pairs(mid, w.potential["cutoff"])
        cnt = ctx.counters()
        assert cnt["limited"] == 0
        if prec == "fp64":
            err = compare_pairs(g, o, w.mean_edge, label="c4")
            log(f"[gpu-c4] fp64: pairs={len(o.dist)} max_rel_err={err:.3e} {cnt}")
        else:
            d_err, t_err = compare32(g, o32, w.mean_edge, "c4")
            log(f"[gpu-c4] fp32: pairs={len(o.dist)} dist_err={d_err:.2e} tan_err={t_err:.2e} {cnt}")
    finally:
        ctx.close()


def test_c4_brownian_step_and_stage_parity(c4, orc):
    """One Brownian step from the initial state against the oracle's step;
    then 20 more GPU steps and a stage-parity check of the pairs on the state
    they reach (bit-exact neighbour sets from the same FP64 state)."""
    from paper_2404_19751_amd import gsim
    w, om, o, _ = c4
    ctx = _ctx("fp64")
    try:
        mid = ctx.mesh_upload(w.mesh.V, w.mesh.T)
        ctx.particles_set(mid, w.face, w.bary)
        p, ig = w.potential, w.integrator
        pot = gsim.potential(p["kind"], p["k"], p["sigma"], p["cutoff"])
        integ = gsim.integrator(ig["kind"], ig["dt"], 1.0, ig["kT"], ig["friction"], ig["seed"])
        log("[gpu-c4] one Brownian step")
        ctx.step(mid, pot, integ, 1)
        fg, bg, _, _ = ctx.particles_get(mid)
        fo, bo, info = orc.step(om, w.face, w.bary, p, ig, 0)
        ok = info["walk_flags"] & 3 == 0
        log(f"[gpu-c4] walk: {info['walk']} unflagged {ok.mean():.4f}")
        assert ok.mean() > 0.99
        assert info["walk"]["boundary_hits"] > 0 and info["walk"]["crossings"] > 10000
        assert np.array_equal(fg[ok], fo[ok])
        assert np.abs(bg[ok] - bo[ok]).max() < 1e-10
        # further steps, then pairs on the GPU's own state against the oracle
        log("[gpu-c4] 20 more steps")
        ctx.step(mid, pot, integ, 20)
        fg, bg, _, _ = ctx.particles_get(mid)
        assert np.all((fg >= 0) & (fg < w.mesh.nf))
        assert np.all(bg >= -1e-12) and np.abs(bg.sum(1) - 1.0).max() < 1e-9
        g = ctx.geodesic_pairs(mid, p["cutoff"])
        o2 = orc.geodesic_pairs(om, fg, bg, p["cutoff"])
        err = compare_pairs(g, o2, w.mean_edge, label="c4-step21")
        log(f"[gpu-c4] stage parity after 21 steps: pairs={len(o2.dist)} err={err:.2e}")
    finally:
        ctx.close()


def test_c4_fp32_step_within_force_bound(c4, orc):
    """One FP32-mixed Brownian step against the oracle's FP64 step, for every
    particle without a near-tie pair: same face, barycentrics within what the
    force tolerance allows (the noise is the same on both sides)."""
    from paper_2404_19751_amd import gsim
    w, om, _, o32 = c4
    ctx = _ctx("fp32")
    try:
        mid = ctx.mesh_upload(w.mesh.V, w.mesh.T)
        ctx.particles_set(mid, w.face, w.bary)
        p, ig = w.potential, w.integrator
        g = ctx.geodesic_pairs(mid, p["cutoff"])
        log("[gpu-c4] fp32: one Brownian step")
        ctx.step(mid, gsim.potential(p["kind"], p["k"], p["sigma"], p["cutoff"]),
                 gsim.integrator(ig["kind"], ig["dt"], 1.0, ig["kT"], ig["friction"], ig["seed"]), 1)
        fg, bg, _, _ = ctx.particles_get(mid)
        fo, bo, info = orc.step(om, w.face, w.bary, p, ig, 0)
        n_cmp, n_same, ratio = step_within_force_bound(w.mesh.V, w.mesh.T, o32, g, p, ig["dt"] / ig["friction"], 1e-5,
                                                       fo, bo, fg, bg, info["walk_flags"])
        log(f"[gpu-c4] fp32 step: {n_cmp} particles compared, {n_same} on the oracle's face, "
            f"barycentric error / bound {ratio:.3f}")
        assert n_cmp > 0.5 * len(w.face) and n_same == n_cmp and ratio <= 1.0
    finally:
        ctx.close()
