"""GPU tests of the batched path: several surfaces stepped by one persistent
geodesic launch and one update launch per step, steps captured in HIP graphs,
and the autotuner.

Batching must not change any result: a surface stepped inside a batch ends in
exactly the state it reaches when stepped alone, and both match the CPU
oracle (faces bit-exact, barycentrics within 1e-11 in FP64 mode)."""
import sys

import numpy as np
import pytest

from paper_2404_19751_amd import workloads as W

pytestmark = pytest.mark.gpu


def log(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _gs():
    from paper_2404_19751_amd import gsim
    return gsim


def small_batch():
    """Four small surfaces of different kinds; the last one Brownian."""
    out = []
    specs = [(W.icosphere(3), 60, 0.45, 11), (W.torus(1.0, 0.3, 30, 12), 80, 0.35, 12),
             (W.bumpy_sphere(3, 0.15), 70, 0.5, 13), (W.height_field(30, 2.0, 5, 2), 120, 0.25, 14)]
    for k, (m, n, cut, seed) in enumerate(specs):
        f, b = W.random_particles(m.nf, n, seed)
        pot = dict(kind="harmonic", k=1.0, sigma=cut, cutoff=cut)
        if k == 3:
            ig = dict(kind="brownian", dt=0.002, kT=0.1, friction=1.0, seed=5)
        else:
            ig = dict(kind="overdamped", dt=0.02, mobility=1.0)
        out.append((m, f, b, pot, ig))
    return out


def to_gsim(pot, ig):
    gs = _gs()
    p = gs.potential(pot["kind"], pot["k"], pot["sigma"], pot["cutoff"])
    if ig["kind"] == "brownian":
        g = gs.integrator("brownian", ig["dt"], 1.0, ig["kT"], ig["friction"], ig["seed"])
    else:
        g = gs.integrator("overdamped", ig["dt"], ig["mobility"])
    return p, g


def load(ctx, batch):
    mids = []
    for m, f, b, _, _ in batch:
        mid = ctx.mesh_upload(m.V, m.T)
        ctx.particles_set(mid, f, b)
        mids.append(mid)
    return mids


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_batched_equals_single(prec):
    """One batched launch per stage gives the same state as stepping each
    surface alone, bit for bit."""
    gs = _gs()
    batch = small_batch()
    cb, cs = gs.Context(0, prec), gs.Context(0, prec)
    try:
        mb, ms = load(cb, batch), load(cs, batch)
        pots, igs = zip(*[to_gsim(p, g) for _, _, _, p, g in batch])
        log(f"[gpu-batch] {prec}: batched 3 steps of {len(batch)} surfaces")
        cb.tune(graph_steps=0)
        cb.step_batched(mb, pots, igs, 3)
        for k, mid in enumerate(ms):
            cs.step(mid, pots[k], igs[k], 3)
        for k in range(len(batch)):
            fb, bb, vb, _ = cb.particles_get(mb[k])
            fs, bs, vs, _ = cs.particles_get(ms[k])
            assert np.array_equal(fb, fs), f"surface {k}: faces differ"
            assert np.array_equal(bb, bs), f"surface {k}: barycentrics differ"
    finally:
        cb.close()
        cs.close()


def test_batched_against_oracle(orc):
    """Two batched FP64 steps (the last surface Brownian: steps 0 and 1 of
    its noise counter) against the oracle's steps of each surface."""
    gs = _gs()
    batch = small_batch()
    ctx = gs.Context(0, "fp64")
    try:
        mids = load(ctx, batch)
        pots, igs = zip(*[to_gsim(p, g) for _, _, _, p, g in batch])
        log("[gpu-batch] batched FP64 vs oracle, 2 steps")
        ctx.step_batched(mids, pots, igs, 2)  # two steps: one graph of 2
        for k, (m, f, b, pot, ig) in enumerate(batch):
            om = orc.OracleMesh(m.V, m.T)
            fo, bo = f, b
            flags = np.zeros(len(f), np.int64)
            for s in range(2):
                fo, bo, info = orc.step(om, fo, bo, pot, ig, s)
                flags |= info["walk_flags"]
            fg, bg, _, _ = ctx.particles_get(mids[k])
            ok = flags & 3 == 0
            assert ok.mean() > 0.97
            assert np.array_equal(fg[ok], fo[ok]), f"surface {k}: faces differ from the oracle"
            assert np.abs(bg[ok] - bo[ok]).max() < 1e-11, f"surface {k}: {np.abs(bg[ok] - bo[ok]).max()}"
    finally:
        ctx.close()


def test_graph_replay_equals_eager():
    """Steps replayed from a captured HIP graph (3 replays of a 4-step graph
    plus one eager step) equal eager steps; the Brownian surface checks that
    the noise counter advances inside the replays."""
    gs = _gs()
    batch = small_batch()
    cg, ce = gs.Context(0, "fp64"), gs.Context(0, "fp64")
    try:
        mg, me = load(cg, batch), load(ce, batch)
        pots, igs = zip(*[to_gsim(p, g) for _, _, _, p, g in batch])
        cg.tune(graph_steps=4)
        ce.tune(graph_steps=0)
        log("[gpu-batch] graph replay vs eager, 13 steps")
        cg.step_batched(mg, pots, igs, 13)
        ce.step_batched(me, pots, igs, 13)
        # a second call reuses the cached graph
        cg.step_batched(mg, pots, igs, 8)
        ce.step_batched(me, pots, igs, 8)
        for k in range(len(batch)):
            fg, bg, vg, _ = cg.particles_get(mg[k])
            fe, be, ve, _ = ce.particles_get(me[k])
            assert np.array_equal(fg, fe) and np.array_equal(bg, be), f"surface {k}"
        assert cg.counters()["cum_pairs"] == ce.counters()["cum_pairs"] > 0
    finally:
        cg.close()
        ce.close()


@pytest.fixture(scope="module")
def c3():
    return W.workload("c3")


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_c3_batch_step(c3, orc, prec):
    """The 16-surface batch (icospheres L3-L6 and 12 tori, 15,033 particles):
    one batched step against the oracle's step of every surface. FP64: faces
    bit-exact, barycentrics within 1e-11. FP32-mixed: the pairs of every
    surface against the oracle's (tie band 1e-5), and the step of every
    particle without a near-tie pair on the oracle's face with barycentrics
    within the force tolerance's bound."""
    gs = _gs()
    ctx = gs.Context(0, prec)
    try:
        mids = load(ctx, [(w.mesh, w.face, w.bary, None, None) for w in c3])
        pots, igs = zip(*[to_gsim(w.potential, w.integrator) for w in c3])
        if prec == "fp64":
            log("[gpu-batch] c3 fp64: one batched step")
            ctx.step_batched(mids, pots, igs, 1)
            assert ctx.counters()["limited"] == 0
            for k, w in enumerate(c3):
                om = orc.OracleMesh(w.mesh.V, w.mesh.T)
                fo, bo, info = orc.step(om, w.face, w.bary, w.potential, w.integrator, 0)
                fg, bg, _, _ = ctx.particles_get(mids[k])
                ok = info["walk_flags"] & 3 == 0
                assert np.array_equal(fg[ok], fo[ok]), f"{w.name}: faces differ"
                assert np.abs(bg[ok] - bo[ok]).max() < 1e-11, w.name
        else:
            from tests.test_gpu_fp32 import compare32
            from tests.util import oracle_band, step_within_force_bound
            gp = []
            for k, w in enumerate(c3):
                om = orc.OracleMesh(w.mesh.V, w.mesh.T)
                g = ctx.geodesic_pairs(mids[k], w.potential["cutoff"])
                o = orc.geodesic_pairs(om, w.face, w.bary, w.potential["cutoff"], **oracle_band("fp32"))
                compare32(g, o, w.mean_edge, w.name)
                gp.append((g, o))
            log("[gpu-batch] c3 fp32: one batched step")
            ctx.step_batched(mids, pots, igs, 1)
            assert ctx.counters()["limited"] == 0
            tot, tot_same, worst = 0, 0, 0.0
            for k, w in enumerate(c3):
                om = orc.OracleMesh(w.mesh.V, w.mesh.T)
                fo, bo, info = orc.step(om, w.face, w.bary, w.potential, w.integrator, 0)
                fg, bg, _, _ = ctx.particles_get(mids[k])
                g, o = gp[k]
                ig = w.integrator
                n_cmp, n_same, ratio = step_within_force_bound(w.mesh.V, w.mesh.T, o, g, w.potential,
                                                               ig["mobility"] * ig["dt"], 1e-5, fo, bo, fg, bg,
                                                               info["walk_flags"])
                assert n_same == n_cmp and ratio <= 1.0, (w.name, n_cmp, n_same, ratio)
                tot, tot_same, worst = tot + n_cmp, tot_same + n_same, max(worst, ratio)
            log(f"[gpu-batch] c3 fp32 step: {tot} particles compared, all on the oracle's face, "
                f"barycentric error / bound {worst:.3f}")
            assert tot > 0.5 * sum(len(w.face) for w in c3)
    finally:
        ctx.close()


def test_autotune_keeps_state_and_results(c3):
    gs = _gs()
    ctx = gs.Context(0, "fp32")
    try:
        sub = c3[:6]
        mids = load(ctx, [(w.mesh, w.face, w.bary, None, None) for w in sub])
        pots, igs = zip(*[to_gsim(w.potential, w.integrator) for w in sub])
        before = [ctx.geodesic_pairs(m, w.potential["cutoff"]) for m, w in zip(mids, sub)]
        log("[gpu-batch] autotune")
        pick = ctx.autotune(mids, pots, igs, reps=2)
        log(f"[gpu-batch] autotune picked {pick}")
        assert pick["lds_stack_kb"] in (4, 8, 16) and pick["update_block"] in (64, 128, 256)
        for k, w in enumerate(sub):
            f, b, _, _ = ctx.particles_get(mids[k])
            assert np.array_equal(f, w.face) and np.array_equal(b, w.bary)
            after = ctx.geodesic_pairs(mids[k], w.potential["cutoff"])
            assert np.array_equal(after["nbr"], before[k]["nbr"])
            assert np.array_equal(after["dist"], before[k]["dist"])
    finally:
        ctx.close()


@pytest.mark.parametrize("kb", [4, 8])
def test_lds_stack_variants(orc, kb):
    """Shallower LDS window stacks (more overflow to global memory) give the
    same pairs as the oracle."""
    gs = _gs()
    w = W.workload("c2")
    ctx = gs.Context(0, "fp64")
    try:
        ctx.tune(lds_stack_kb=kb, grab=2)
        mid = ctx.mesh_upload(w.mesh.V, w.mesh.T)
        ctx.particles_set(mid, w.face, w.bary)
        g = ctx.geodesic_pairs(mid, w.potential["cutoff"])
        om = orc.OracleMesh(w.mesh.V, w.mesh.T)
        o = orc.geodesic_pairs(om, w.face, w.bary, w.potential["cutoff"])
        from tests.test_gpu_parity import compare_pairs
        err = compare_pairs(g, o, w.mean_edge, label=f"c2-lds{kb}")
        log(f"[gpu-batch] lds_stack_kb={kb}: err {err:.2e}")
    finally:
        ctx.close()
