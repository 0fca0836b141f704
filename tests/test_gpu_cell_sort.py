"""The cell counting sort of a surface whose grid is too fine for one
workgroup (the height field, 20,000 particles): its counts start from zeros
and the scatter leaves zeros behind, so passes need no clearing kernel. Runs
on one context with grids of different sizes in turn (a finer grid than any
before, a coarser one, then the finer one again without a clear), each
checked against the oracle: neighbour sets bit-exact, distances and
tangents within 1e-12."""
import sys

import numpy as np
import pytest

from paper_2404_19751_amd import workloads as W
from tests.test_gpu_parity import compare_pairs

pytestmark = pytest.mark.gpu


def log(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def test_cell_sort_across_grid_sizes(orc):
    from paper_2404_19751_amd import gsim
    w = W.workload("c4")
    om = orc.OracleMesh(w.mesh.V, w.mesh.T)
    cut = w.potential["cutoff"]
    cuts = [0.6 * cut, cut, 0.6 * cut]
    ref = {c: orc.geodesic_pairs(om, w.face, w.bary, c) for c in set(cuts)}
    ctx = gsim.Context(0, "fp64")
    try:
        mid = ctx.mesh_upload(w.mesh.V, w.mesh.T)
        ctx.particles_set(mid, w.face, w.bary)
        for k, c in enumerate(cuts):
            log(f"[gpu-cell-sort] pass {k} cutoff {c:.5f}")
            g = ctx.geodesic_pairs(mid, c)
            assert ctx.counters()["limited"] == 0
            err = compare_pairs(g, ref[c], w.mean_edge, label=f"cell-sort-{k}")
            log(f"[gpu-cell-sort] pass {k}: pairs={len(ref[c].dist)} max_rel_err={err:.3e}")
            assert err <= 1e-12
    finally:
        ctx.close()
