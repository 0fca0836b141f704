"""Two or four sources per wavefront (the grouped instantiations of the
cutoff kernel: FP64 passes with more sources than resident wavefronts)
against one source per wavefront, on the height field (20,000 sources) and the 16 batched
surfaces of C3: the same neighbour rows and flags, distances and tangents
equal to rounding (the two instantiations are compiled separately, so their
multiply-adds may be contracted differently), and the same steps."""
import sys

import numpy as np
import pytest

from paper_2404_19751_amd import workloads as W

pytestmark = pytest.mark.gpu


def log(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _pairs_and_steps(ws, group, steps):
    from paper_2404_19751_amd import gsim
    ctx = gsim.Context(0, "fp64")
    try:
        ctx.tune(group_sources=group)
        mids = []
        for w in ws:
            mid = ctx.mesh_upload(w.mesh.V, w.mesh.T)
            ctx.particles_set(mid, w.face, w.bary)
            mids.append(mid)
        rows = [ctx.geodesic_pairs(mid, w.potential["cutoff"]) for mid, w in zip(mids, ws)]
        cnt = ctx.counters()
        assert cnt["limited"] == 0
        pots = [gsim.potential(w.potential["kind"], w.potential["k"], w.potential["sigma"], w.potential["cutoff"])
                for w in ws]
        igs = [gsim.integrator(w.integrator["kind"], w.integrator["dt"], **{k: v for k, v in w.integrator.items()
                                                                           if k not in ("kind", "dt")})
               for w in ws]
        if len(ws) == 1:
            ctx.step(mids[0], pots[0], igs[0], steps)
        else:
            ctx.step_batched(mids, pots, igs, steps)
        states = [ctx.particles_get(mid) for mid in mids]
        return rows, states, cnt
    finally:
        ctx.close()


@pytest.mark.parametrize("group", [2, 4])
@pytest.mark.parametrize("name", ["c4", "c3"])
def test_groups_equal_single_sources(name, group):
    ws = W.workload(name)
    ws = ws if isinstance(ws, list) else [ws]
    log(f"[gpu-pairs] {name}: {sum(len(w.face) for w in ws)} sources, one and {group} per wavefront")
    r1, s1, c1 = _pairs_and_steps(ws, 1, 3)
    r2, s2, c2 = _pairs_and_steps(ws, group, 3)
    worst = 0.0
    for a, b in zip(r1, r2):
        assert np.array_equal(a["off"], b["off"]) and np.array_equal(a["nbr"], b["nbr"])
        assert np.array_equal(a["flags"], b["flags"])
        if len(a["dist"]):
            rel = np.abs(a["dist"] - b["dist"]) / np.maximum(a["dist"], 1e-300)
            dt = np.linalg.norm(a["tan"] - b["tan"], axis=1)
            worst = max(worst, float(rel.max()), float(dt.max()))
    assert worst <= 1e-13
    same = total = 0
    bmax = 0.0
    for a, b in zip(s1, s2):
        eq = a[0] == b[0]
        same += int(eq.sum())
        total += len(eq)
        if eq.any():
            bmax = max(bmax, float(np.abs(a[1][eq] - b[1][eq]).max()))
    assert same >= total - 2 and bmax <= 1e-11
    log(f"[gpu-pairs] {name}: rows equal, distances and tangents within {worst:.1e}; after 3 steps {same} of "
        f"{total} particles on the same face, barycentrics within {bmax:.1e}; windows {c1['windows']} (one) / "
        f"{c2['windows']} ({group} per wavefront)")
