"""GPU parity on the meshes of the fixed-N mesh-size sweep (N = 100, range
one tenth of the span): the sphere, and tori of aspect ratio 3 and 20.
Submeshed passes (cutoff = range) on every pair against the oracle;
full-mesh passes (no cutoff) on sampled source rows."""
import math
import sys

import numpy as np
import pytest

from paper_2404_19751_amd import workloads as W
from tests.test_gpu_parity import compare_pairs

pytestmark = pytest.mark.gpu


def log(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.mark.parametrize("name", ["vsweep_sphere_4", "vsweep_torus3_24", "vsweep_torus20_8"])
def test_vsweep_submesh(orc, name):
    from paper_2404_19751_amd import gsim
    w = W.workload(name)
    cut = w.potential["cutoff"]
    ctx = gsim.Context(0, "fp64")
    try:
        mid = ctx.mesh_upload(w.mesh.V, w.mesh.T)
        ctx.particles_set(mid, w.face, w.bary)
        log(f"[gpu-vsweep] {name}: submesh, cutoff {cut}")
        g = ctx.geodesic_pairs(mid, cut)
        o = orc.geodesic_pairs(orc.OracleMesh(w.mesh.V, w.mesh.T), w.face, w.bary, cut)
        err = compare_pairs(g, o, w.mean_edge, label=name)
        log(f"[gpu-vsweep] {name}: {len(o.dist)} pairs, err {err:.2e}")
    finally:
        ctx.close()


@pytest.mark.parametrize("name,srcs", [("vsweep_sphere_4", [0, 50, 99]), ("vsweep_torus3_17", [0, 37, 99]),
                                       ("vsweep_torus20_6", [0, 99])])
def test_vsweep_full_mesh_rows(orc, name, srcs):
    from paper_2404_19751_amd import gsim
    w = W.workload(name)
    ctx = gsim.Context(0, "fp64")
    try:
        mid = ctx.mesh_upload(w.mesh.V, w.mesh.T)
        ctx.particles_set(mid, w.face, w.bary)
        log(f"[gpu-vsweep] {name}: full mesh")
        g = ctx.geodesic_pairs(mid, math.inf)
        assert ctx.counters()["limited"] == 0
        s = np.array(srcs, np.int32)
        o = orc.geodesic_pairs(orc.OracleMesh(w.mesh.V, w.mesh.T), w.face, w.bary, math.inf, sources=s)
        sub = {"off": [0], "nbr": [], "dist": [], "tan": [], "flags": []}
        for i in s:
            a, b = g["off"][i], g["off"][i + 1]
            for key in ("nbr", "dist", "tan", "flags"):
                sub[key].append(g[key][a:b])
            sub["off"].append(sub["off"][-1] + b - a)
        gs = {k: (np.concatenate(v) if k != "off" else np.array(v, np.int64)) for k, v in sub.items()}
        err = compare_pairs(gs, o, w.mean_edge, label=name)
        log(f"[gpu-vsweep] {name}: full-mesh rows err {err:.2e}")
    finally:
        ctx.close()
