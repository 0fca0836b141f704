"""The allocation-free walk (gsim_displace_on_surface_noalloc) through the
C ABI against gsim_displace_on_surface_dev: two calls in a row, the second
on a smaller input, each bit-identical in particle state, per-particle flags
and walk statistics (the shift of Sec. 3.2); and the particle limit of its
scratch array."""
import sys

import numpy as np
import pytest

from paper_2404_19751_amd import workloads as W

pytestmark = pytest.mark.gpu


def log(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _walk_both(torch, gs, ctx, w, D, vel):
    """The same walk through the allocating and the allocation-free entry
    point, from the same state; returns both results."""
    n = len(w.face)
    mid = ctx.mesh_upload(w.mesh.V, w.mesh.T)
    D_t = torch.tensor(D, dtype=torch.float64, device="cuda")
    out = []
    for noalloc in (False, True):
        ctx.particles_set(mid, w.face, w.bary, vel)
        torch.cuda.synchronize()
        if noalloc:
            fl_t = torch.full((n,), 255, dtype=torch.uint8, device="cuda")
            torch.cuda.synchronize()
            st = ctx.displace_on_surface_noalloc(mid, D_t, fl_t)
            fl = fl_t.cpu().numpy()
        else:
            st = ctx.displace_on_surface_dev(mid, D_t)
            fl = ctx.particle_flags(mid)
        f, b, v, _ = ctx.particles_get(mid)
        out.append((st, fl, f, b, v))
    return out


def test_noalloc_walk_matches_dev_walk_twice():
    import torch
    from paper_2404_19751_amd import gsim as gs
    ctx = gs.Context(0, "fp64")
    try:
        # first call: 20,000 particles on the open height field (boundary
        # reflections, crossings); second: 64 on the small sphere
        for name, scale in (("c4", 0.08), ("c1", 0.05)):
            w = W.workload(name)
            n = len(w.face)
            rng = np.random.default_rng(12)
            D = scale * rng.normal(size=(n, 3))
            vel = rng.normal(size=(n, 3))
            log(f"[no-alloc] {name}: {n} particles")
            (sa, fa, f1, b1, v1), (sb, fb, f2, b2, v2) = _walk_both(torch, gs, ctx, w, D, vel)
            assert sa == sb, (sa, sb)
            assert np.array_equal(fa, fb)
            assert np.array_equal(f1, f2) and np.array_equal(b1, b2) and np.array_equal(v1, v2)
            assert sa["crossings"] > 0
            log(f"[no-alloc] {name}: identical, stats {sb}")
    finally:
        ctx.close()


def test_noalloc_walk_limit():
    """More particles than the scratch array serves: a limit error, and the
    state is not touched."""
    import torch
    from paper_2404_19751_amd import gsim as gs
    m = W.icosphere(3)
    n = 2_097_153
    f, b = W.random_particles(m.nf, n, 5)
    ctx = gs.Context(0, "fp64")
    try:
        mid = ctx.mesh_upload(m.V, m.T)
        ctx.particles_set(mid, f, b)
        D_t = torch.zeros((n, 3), dtype=torch.float64, device="cuda")
        torch.cuda.synchronize()
        with pytest.raises(gs.GsimError) as e:
            ctx.displace_on_surface_noalloc(mid, D_t)
        assert e.value.status == gs.E_LIMIT and "2097152" in str(e.value)
        log("[no-alloc] limit reported")
    finally:
        ctx.close()
