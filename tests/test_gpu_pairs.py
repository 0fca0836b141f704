"""Two, four or eight sources per wavefront (the grouped instantiations of
the cutoff kernel: passes with more sources than resident wavefronts)
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


@pytest.mark.parametrize("group", [2, 4, 8])
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


def _clustered_c4():
    """The height field's particles plus a seeded cluster of 60 within 0.45
    cutoff of particle 0: about 70 sources then have 33-72 candidates, more
    than a group's share (32), while the mean stays near 7.5."""
    w = W.workload("c4")
    cut = w.potential["cutoff"]
    x0 = w.bary[0] @ w.mesh.V[w.mesh.T[w.face[0]]]
    cent = w.mesh.V[w.mesh.T].mean(1)
    near = np.nonzero(np.linalg.norm(cent - x0, axis=1) < 0.45 * cut)[0]
    rng = np.random.default_rng(5)
    fc = near[rng.integers(0, len(near), 60)].astype(np.int32)
    u1, u2 = rng.random(60), rng.random(60)
    bc = np.stack([1 - np.sqrt(u1), np.sqrt(u1) * (1 - u2), np.sqrt(u1) * u2], 1)
    return w, np.concatenate([w.face, fc]), np.concatenate([w.bary, bc]), cut


def test_group_sources_with_too_many_candidates_run_alone(orc):
    """Sources with more candidates than a group's share of the table run
    alone over the whole table: the rows equal those of one source per
    wavefront, and the crowded sources' rows match the oracle."""
    from paper_2404_19751_amd import gsim
    from tests.test_gpu_parity import compare_pairs
    w, face, bary, cut = _clustered_c4()
    out = {}
    for group in (1, 4):
        ctx = gsim.Context(0, "fp64")
        try:
            ctx.tune(group_sources=group)
            mid = ctx.mesh_upload(w.mesh.V, w.mesh.T)
            ctx.particles_set(mid, face, bary)
            out[group] = ctx.geodesic_pairs(mid, cut)
            assert ctx.counters()["limited"] == 0
        finally:
            ctx.close()
    a, b = out[1], out[4]
    assert np.array_equal(a["off"], b["off"]) and np.array_equal(a["nbr"], b["nbr"])
    assert np.array_equal(a["flags"], b["flags"])
    assert np.abs(a["dist"] - b["dist"]).max() <= 1e-13 * a["dist"].max()
    crowded = np.nonzero(np.diff(b["off"]) > 32)[0]
    assert len(crowded) >= 20
    src = np.concatenate([crowded, np.arange(0, 20000, 997)]).astype(np.int32)
    om = orc.OracleMesh(w.mesh.V, w.mesh.T)
    o = orc.geodesic_pairs(om, face, bary, cut, sources=src)
    sub = {k: np.concatenate([b[k][b["off"][i]:b["off"][i + 1]] for i in src]) for k in ("nbr", "dist", "tan", "flags")}
    sub["off"] = np.concatenate([[0], np.cumsum([b["off"][i + 1] - b["off"][i] for i in src])])
    err = compare_pairs(sub, o, w.mean_edge, label="clustered c4")
    log(f"[gpu-pairs] clustered c4: {len(crowded)} sources with more than 32 candidates ran alone; "
        f"{len(o.dist)} sampled pairs against the oracle, err {err:.2e}")


def test_fp32_groups_against_oracle(orc):
    """FP32-mixed with four sources per wavefront on the clustered height
    field: the group in FP32, sources with a pair in the guard band again
    alone in FP64, crowded sources alone. Their rows and a sample of the rest
    match the oracle to the FP32 tolerance (bit-exact neighbour sets)."""
    from paper_2404_19751_amd import gsim
    from tests.test_gpu_fp32 import compare32
    from tests.util import oracle_band
    w, face, bary, cut = _clustered_c4()
    ctx = gsim.Context(0, "fp32")
    try:
        ctx.tune(group_sources=4)
        mid = ctx.mesh_upload(w.mesh.V, w.mesh.T)
        ctx.particles_set(mid, face, bary)
        b = ctx.geodesic_pairs(mid, cut)
        cnt = ctx.counters()
        assert cnt["limited"] == 0
    finally:
        ctx.close()
    crowded = np.nonzero(np.diff(b["off"]) > 32)[0]
    assert len(crowded) >= 20
    guard = np.nonzero(np.bitwise_and(b["flags"], 4))[0]
    gsrc = np.unique(np.searchsorted(b["off"], guard, side="right") - 1)
    src = np.unique(np.concatenate([crowded, gsrc[:40], np.arange(0, 20000, 997)])).astype(np.int32)
    om = orc.OracleMesh(w.mesh.V, w.mesh.T)
    o = orc.geodesic_pairs(om, face, bary, cut, sources=src, **oracle_band("fp32"))
    sub = {k: np.concatenate([b[k][b["off"][i]:b["off"][i + 1]] for i in src]) for k in ("nbr", "dist", "tan", "flags")}
    sub["off"] = np.concatenate([[0], np.cumsum([b["off"][i + 1] - b["off"][i] for i in src])])
    d_err, t_err = compare32(sub, o, w.mean_edge, "clustered c4 fp32")
    log(f"[gpu-pairs] clustered c4 fp32: {len(crowded)} crowded sources, {len(gsrc)} recomputed in FP64 "
        f"({cnt['guard_sources']} guard runs); {len(src)} sources against the oracle, dist err {d_err:.2e}, "
        f"tan err {t_err:.2e}")
