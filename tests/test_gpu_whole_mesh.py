"""GPU parity of finite-cutoff passes on the whole-mesh kernel (the
"whole_mesh" knob): rows of every target, windows pruned at the cutoff, no
per-source limit on candidates or bend vertices. Checked against the CPU
oracle on a saddle-rich torus, against the cutoff kernel on the bumpy
sphere (both exact, so they must agree), and at cutoffs a hair above and
below a true pair distance in FP32-mixed mode (FP64 recompute)."""
import math
import sys

import numpy as np
import pytest

from paper_2404_19751_amd import workloads as W
from tests.test_gpu_fp32 import compare32
from tests.util import oracle_band
from tests.test_gpu_parity import compare_pairs

pytestmark = pytest.mark.gpu


def log(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _ctx(prec, whole):
    from paper_2404_19751_amd import gsim
    c = gsim.Context(0, prec)
    c.tune(whole_mesh=1 if whole else 0)
    return c


@pytest.fixture(scope="module")
def torus_case(orc):
    m = W.torus(3.0, 1.0, 48, 16)
    f, b = W.random_particles(m.nf, 300, 37)
    cut = 5.0
    om = orc.OracleMesh(m.V, m.T)
    o = orc.geodesic_pairs(om, f, b, cut)
    o32 = orc.geodesic_pairs(om, f, b, cut, **oracle_band("fp32"))
    return m, f, b, cut, o, o32


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_whole_mesh_cutoff_matches_oracle(torus_case, prec):
    m, f, b, cut, o, o32 = torus_case
    ctx = _ctx(prec, True)
    try:
        mid = ctx.mesh_upload(m.V, m.T)
        ctx.particles_set(mid, f, b)
        log(f"[gpu-whole] torus a3 {prec}: cutoff {cut}, {len(f)} particles")
        g = ctx.geodesic_pairs(mid, cut)
        cnt = ctx.counters()
        assert cnt["limited"] == 0
        assert np.diff(o.off).max() > 128  # more neighbours than the cutoff kernel's LDS table holds
        if prec == "fp64":
            err = compare_pairs(g, o, W.mean_edge_length(m), label="torus_a3")
        else:
            err, _ = compare32(g, o32, W.mean_edge_length(m), "torus_a3")
        log(f"[gpu-whole] torus a3 {prec}: {len(o.dist)} pairs, err {err:.2e}, counters {cnt}")
    finally:
        ctx.close()


def test_cutoff_kernel_takes_wide_patches(torus_case):
    """The same case on the cutoff kernel, whose sources have more candidates
    than its LDS table holds: the big-candidate instantiation matches the
    oracle too."""
    m, f, b, cut, o, _ = torus_case
    ctx = _ctx("fp64", False)
    try:
        mid = ctx.mesh_upload(m.V, m.T)
        ctx.particles_set(mid, f, b)
        g = ctx.geodesic_pairs(mid, cut)
        assert ctx.counters()["limited"] == 0
        err = compare_pairs(g, o, W.mean_edge_length(m), label="torus_a3 cutoff kernel")
        log(f"[gpu-whole] torus a3 on the cutoff kernel: {len(o.dist)} pairs, err {err:.2e}")
    finally:
        ctx.close()


def test_cutoff_kernel_reports_its_limit():
    """More Euclidean candidates per source than the big-candidate kernel
    takes (4096): a limit error naming the whole-mesh knob, not a partial
    result."""
    from paper_2404_19751_amd import gsim
    m = W.icosphere(3)
    f, b = W.random_particles(m.nf, 5000, 3)
    ctx = _ctx("fp64", False)
    try:
        mid = ctx.mesh_upload(m.V, m.T)
        ctx.particles_set(mid, f, b)
        with pytest.raises(gsim.GsimError) as e:
            ctx.geodesic_pairs(mid, 3.0)
        assert e.value.status == gsim.E_LIMIT
        assert "whole_mesh" in str(e.value)
    finally:
        ctx.close()


def test_whole_mesh_rows_checked_against_free_memory():
    """46,000 particles need 78 GB of whole-mesh rows (37 bytes a pair
    slot): with most of the device held by a torch allocation first, the
    pass is refused with GSIM_E_LIMIT naming the bytes, before any row is
    allocated; once the memory is back the same context runs a small pass."""
    import torch
    from paper_2404_19751_amd import gsim
    m = W.icosphere(5)
    n = 46000
    f, b = W.random_particles(m.nf, n, 9)
    free, total = torch.cuda.mem_get_info()
    hold_bytes = max(0, free - 40 * 2**30)  # leave 40 GB: less than the rows need
    log(f"[gpu-whole] holding {hold_bytes / 2**30:.0f} GiB of {total / 2**30:.0f} GiB")
    hold = torch.empty(hold_bytes, dtype=torch.uint8, device="cuda")
    ctx = _ctx("fp64", True)
    try:
        mid = ctx.mesh_upload(m.V, m.T)
        ctx.particles_set(mid, f, b)
        with pytest.raises(gsim.GsimError) as e:
            ctx.geodesic_pairs(mid, 0.05)
        assert e.value.status == gsim.E_LIMIT
        assert "46000 particles" in str(e.value) and "GB" in str(e.value)
        del hold
        torch.cuda.empty_cache()
        ctx.particles_set(mid, f[:500], b[:500])
        g = ctx.geodesic_pairs(mid, 0.05)
        assert len(g["nbr"]) > 0
    finally:
        ctx.close()


def test_whole_mesh_agrees_with_cutoff_kernel():
    """Bumpy sphere, 1000 particles, cutoff 0.15: the whole-mesh kernel and
    the cutoff kernel are both exact, so neighbour sets are identical and
    distances and tangents agree to rounding; so do forces and a few steps."""
    from paper_2404_19751_amd import gsim
    w = W.workload("c2")
    pot = gsim.potential("harmonic", 1.0, 0.15, 0.15)
    ig = gsim.integrator("overdamped", 0.01)
    out = {}
    for whole in (False, True):
        ctx = _ctx("fp64", whole)
        try:
            mid = ctx.mesh_upload(w.mesh.V, w.mesh.T)
            ctx.particles_set(mid, w.face, w.bary)
            log(f"[gpu-whole] c2 whole_mesh={whole}")
            g = ctx.geodesic_pairs(mid, 0.15)
            F, E = ctx.compute_forces(mid, pot)
            ctx.step(mid, pot, ig, 5)
            f, b, _, _ = ctx.particles_get(mid)
            out[whole] = (g, F, E, f, b)
        finally:
            ctx.close()
    (g0, F0, E0, f0, b0), (g1, F1, E1, f1, b1) = out[False], out[True]
    assert np.array_equal(g0["off"], g1["off"]) and np.array_equal(g0["nbr"], g1["nbr"])
    assert np.abs(g0["dist"] - g1["dist"]).max() <= 1e-12 * g0["dist"].max()
    tie = ((g0["flags"] & 1) != 0) | ((g1["flags"] & 1) != 0)
    assert np.abs(g0["tan"] - g1["tan"])[~tie].max() <= 1e-9
    assert abs(E0 - E1) <= 1e-12 * abs(E0)
    assert np.abs(F0 - F1).max() <= 1e-10 * np.abs(F0).max()
    assert np.array_equal(f0, f1) and np.abs(b0 - b1).max() <= 1e-10
    log(f"[gpu-whole] c2: {len(g0['dist'])} pairs agree; forces and 5 steps agree")


def test_whole_mesh_fp32_guard_band(torus_case, orc):
    """Cutoffs a hair above and below a true pair distance in FP32-mixed
    mode: the FP64 recompute decides membership exactly as the oracle does."""
    m, f, b, cut, o, _ = torus_case
    om = orc.OracleMesh(m.V, m.T)
    d = float(np.sort(o.dist)[len(o.dist) // 2])
    ctx = _ctx("fp32", True)
    try:
        mid = ctx.mesh_upload(m.V, m.T)
        ctx.particles_set(mid, f, b)
        for c in (d * (1 + 3e-9), d * (1 - 3e-9)):
            log(f"[gpu-whole] guard band: cutoff {c!r}")
            g = ctx.geodesic_pairs(mid, c)
            oo = orc.geodesic_pairs(om, f, b, c)
            assert np.array_equal(g["off"], oo.off) and np.array_equal(g["nbr"], oo.nbr)
            assert (g["flags"] & 4).any()
            assert ctx.counters()["guard_sources"] >= 1
    finally:
        ctx.close()
