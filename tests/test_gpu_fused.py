"""The fused time step, where the cutoff kernel moves each source particle as
soon as its row is final and the next step's binning (or a commit launch
after the last step) makes the next state current, against the separate
update launch: trajectories are bit-identical for every integrator it covers
(overdamped, Brownian, velocity Verlet), in both precision modes, eagerly and
through cached HIP graph replays, for one surface and for a batch. Fusion is
taken only with at most four particles per compute unit (one source per
SIMD); each case checks that it was."""
import copy
import sys

import numpy as np
import pytest

from paper_2404_19751_amd import workloads as W

pytestmark = pytest.mark.gpu


def log(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def args(gs, w):
    p, ig = w.potential, w.integrator
    pot = gs.potential(p["kind"], p["k"], p["sigma"], p["cutoff"])
    if ig["kind"] == "brownian":
        integ = gs.integrator("brownian", ig["dt"], 1.0, ig["kT"], ig["friction"], ig["seed"])
    elif ig["kind"] == "overdamped":
        integ = gs.integrator("overdamped", ig["dt"], ig["mobility"])
    else:
        integ = gs.integrator(ig["kind"], ig["dt"])
    return pot, integ


def run(ws, prec, fuse, chunks):
    """Steps of the surfaces `ws` (batched when more than one) in calls of
    `chunks` steps each; the final states and the pair count."""
    from paper_2404_19751_amd import gsim as gs
    ctx = gs.Context(0, prec)
    try:
        ctx.tune(fuse_update=fuse)
        mids = []
        for w in ws:
            mid = ctx.mesh_upload(w.mesh.V, w.mesh.T)
            ctx.particles_set(mid, w.face, w.bary)
            mids.append(mid)
        pots, igs = zip(*[args(gs, w) for w in ws])
        # one timed (eager) step tells whether the step was fused: a fused
        # call ends with one commit launch
        ctx.timing(True)
        if len(ws) == 1:
            ctx.step(mids[0], pots[0], igs[0], 1)
        else:
            ctx.step_batched(mids, pots, igs, 1)
        commits = ctx.timing_get("commit")[1]
        ctx.timing(False)
        assert commits == (1 if fuse else 0)
        pairs = 0
        for k in chunks:
            if len(ws) == 1:
                ctx.step(mids[0], pots[0], igs[0], k)
            else:
                ctx.step_batched(mids, pots, igs, k)
            assert ctx.counters()["limited"] == 0
            pairs += ctx.counters()["nbr_pairs"]
        return [ctx.particles_get(m)[:3] for m in mids], pairs
    finally:
        ctx.close()


def c4_subset(n=1000):
    """The height field with the first n particles of its workload (Brownian
    dynamics with few enough particles to be fused)."""
    w = copy.copy(W.workload("c4"))
    w.face, w.bary = w.face[:n].copy(), w.bary[:n].copy()
    return w


CASES = [
    ("c2", "fp64", [1, 4, 3]),
    ("c2", "fp32", [1, 4, 3]),
    ("c4_1000", "fp64", [2, 3]),
    ("c4_1000", "fp32", [2, 3]),
    ("torus_nve_1024_0.25", "fp64", [1, 5]),
    ("torus_nve_1024_0.25", "fp32", [1, 5]),
]


@pytest.mark.parametrize("name,prec,chunks", CASES)
def test_fused_step_is_bit_identical(name, prec, chunks):
    w = c4_subset() if name == "c4_1000" else W.workload(name)
    log(f"[gpu-fused] {name} {prec}: steps {chunks}, fused and separate")
    a, pa = run([w], prec, 1, chunks)
    b, pb = run([w], prec, 0, chunks)
    for x, y in zip(a[0], b[0]):
        assert np.array_equal(x, y)
    assert pa == pb
    moved = np.mean(a[0][0] != w.face)
    log(f"[gpu-fused] {name} {prec}: identical; {moved:.3f} of the particles changed face")


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_fused_batched_graph_is_bit_identical(prec):
    # five surfaces with 1010 particles in all (fused); the whole batch
    # (15,033 particles) is not
    ws = [W.workload("c3")[k] for k in (0, 1, 4, 5, 6)]
    log(f"[gpu-fused] c3 subset {prec}: batched, graph replays")
    a, pa = run(ws, prec, 1, [1, 8, 2])
    b, pb = run(ws, prec, 0, [1, 8, 2])
    for sa, sb in zip(a, b):
        for x, y in zip(sa, sb):
            assert np.array_equal(x, y)
    assert pa == pb
