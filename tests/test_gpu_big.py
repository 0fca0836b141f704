"""The cutoff kernel with more Euclidean candidates per source than its LDS
target table holds (the paper's NVE benchmark torus at interaction range
sigma = 1 and 1/2, Sec. 4, Fig. 3): the big-candidate instantiation keeps
each source's targets in global memory and sizes its rows from a device
count of the candidates. Pairs against the oracle in both precisions, one
velocity-Verlet step against the oracle's, the fused update against the
separate one, and agreement with the whole-mesh kernel."""
import sys

import numpy as np
import pytest

from paper_2404_19751_amd import workloads as W
from tests.test_gpu_fp32 import compare32
from tests.test_gpu_parity import compare_pairs
from tests.util import oracle_band

pytestmark = pytest.mark.gpu


def log(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _gs():
    from paper_2404_19751_amd import gsim
    return gsim


def max_candidates(w):
    """The largest number of particles within the cutoff (3D) of a particle."""
    T = w.mesh.T[w.face]
    x = np.einsum("nk,nkd->nd", w.bary, w.mesh.V[T])
    c2 = w.potential["cutoff"] ** 2
    best = 0
    for a in range(0, len(x), 1024):
        d2 = ((x[a:a + 1024, None, :] - x[None, :, :]) ** 2).sum(-1)
        best = max(best, int(((d2 < c2).sum(1) - 1).max()))
    return best


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
@pytest.mark.parametrize("n,sig,big", [(2048, 1.0, False), (8192, 1.0, True), (8192, 0.5, False)])
def test_big_pairs_match_oracle(orc, n, sig, big, prec):
    """Pairs at the cutoff sigma against the oracle; the cases with at most
    128 candidates per source run on the LDS table after the count."""
    gs = _gs()
    w = W.workload(f"torus_nve_{n}_{sig}")
    mc = max_candidates(w)
    log(f"[gpu-big] torus n={n} sigma={sig} {prec}: at most {mc} Euclidean candidates per source")
    om = orc.OracleMesh(w.mesh.V, w.mesh.T)
    o = orc.geodesic_pairs(om, w.face, w.bary, sig, **oracle_band(prec))
    ctx = gs.Context(0, prec)
    try:
        mid = ctx.mesh_upload(w.mesh.V, w.mesh.T)
        ctx.particles_set(mid, w.face, w.bary)
        g = ctx.geodesic_pairs(mid, sig)
        cnt = ctx.counters()
        assert cnt["limited"] == 0
        if prec == "fp64":
            err = compare_pairs(g, o, w.mean_edge, label=f"torus{n}_{sig}")
        else:
            err, _ = compare32(g, o, w.mean_edge, f"torus{n}_{sig}")
        log(f"[gpu-big] n={n} sigma={sig} {prec}: {len(o.dist)} pairs, err {err:.2e}, windows {cnt['windows']}")
    finally:
        ctx.close()
    assert (mc > 128) == big  # which instantiation the count chose


def test_big_verlet_step_matches_oracle(orc):
    """One velocity-Verlet step at sigma = 1, N = 8192 from rest, against
    the oracle's (stage parity: faces bit-exact, barycentrics within 1e-11)."""
    gs = _gs()
    w = W.workload("torus_nve_8192_1.0")
    p = w.potential
    ctx = gs.Context(0, "fp64")
    try:
        mid = ctx.mesh_upload(w.mesh.V, w.mesh.T)
        ctx.particles_set(mid, w.face, w.bary)
        log("[gpu-big] one Verlet step, n=8192 sigma=1")
        ctx.step(mid, gs.potential("harmonic", p["k"], p["sigma"], p["cutoff"]), gs.integrator("verlet", 0.005), 1)
        fg, bg, vg, _ = ctx.particles_get(mid)
        om = orc.OracleMesh(w.mesh.V, w.mesh.T)
        fo, bo, vo, info = orc.verlet_step(om, w.face, w.bary, np.zeros((len(w.face), 3)), p, dict(dt=0.005))
        ok = info["walk_flags"] & 3 == 0
        assert ok.mean() > 0.99
        assert np.array_equal(fg[ok], fo[ok])
        assert np.abs(bg[ok] - bo[ok]).max() < 1e-11
        assert np.abs(vg[ok] - vo[ok]).max() < 1e-11 * max(1.0, np.abs(vo).max())
    finally:
        ctx.close()


def test_big_fused_equals_separate_and_whole_mesh():
    """N = 1000 at sigma = 2 (more than 128 candidates, at most four
    particles per compute unit): the fused update equals the separate one bit
    for bit over several steps, and the pairs equal the whole-mesh kernel's."""
    gs = _gs()
    w = W.workload("torus_nve_1000_2.0")
    assert max_candidates(w) > 128
    p = w.potential
    pot = gs.potential("harmonic", p["k"], p["sigma"], p["cutoff"])
    ig = gs.integrator("verlet", 0.005)
    out = {}
    for mode in ("fused", "separate", "whole"):
        ctx = gs.Context(0, "fp64")
        try:
            ctx.tune(fuse_update=1 if mode == "fused" else 0, whole_mesh=1 if mode == "whole" else 0)
            mid = ctx.mesh_upload(w.mesh.V, w.mesh.T)
            ctx.particles_set(mid, w.face, w.bary)
            g = ctx.geodesic_pairs(mid, p["cutoff"])
            log(f"[gpu-big] n=1000 sigma=2 {mode}: {len(g['nbr'])} pairs; 6 steps")
            ctx.step(mid, pot, ig, 6)
            out[mode] = (g, ctx.particles_get(mid))
            assert ctx.counters()["limited"] == 0
        finally:
            ctx.close()
    gf, (f1, b1, v1, _) = out["fused"]
    gsep, (f2, b2, v2, _) = out["separate"]
    assert np.array_equal(f1, f2) and np.array_equal(b1, b2) and np.array_equal(v1, v2)
    gw, _ = out["whole"]
    assert np.array_equal(gf["off"], gw["off"]) and np.array_equal(gf["nbr"], gw["nbr"])
    assert np.abs(gf["dist"] - gw["dist"]).max() <= 1e-12 * gf["dist"].max()
