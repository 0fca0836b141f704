"""The error of every hot-path result against the FP64 oracle, stated per
workload and precision mode: neighbour sets (bit-exact), distances (relative
error), initial tangents (the log-map vector d*t, relative to
max(d, 1e-3 of the mean edge); pairs flagged as near-ties are measured
against the nearest direction of the oracle's tie set), forces (|dF_i|
relative to sum_j (|U'(d_ij)| + d_ij |U''(d_ij)|), what the per-pair bounds
imply to first order: over particles without a near-tie pair, whose force
may legitimately take either direction, and over all particles with the
GPU's direction taken for tie pairs), the energy, and one step's faces and
barycentric coordinates (particles whose walk the oracle flags as passing
within the hit tolerance of a vertex or edge excluded).

Each case prints one `[error-report]` JSON line and asserts the bounds: 1e-12
(FP64; forces 1e-11) and 1e-5 (FP32-mixed) relative."""
import json
import math
import sys

import numpy as np
import pytest

from paper_2404_19751_amd import workloads as W
from tests.util import force_scale, oracle_band, step_within_force_bound, tangent_errors

pytestmark = pytest.mark.gpu
RTOL = {"fp64": 1e-12, "fp32": 1e-5}
FTOL = {"fp64": 1e-11, "fp32": 1e-5}


def log(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def pair_errors(g, o, lbar):
    """Exact neighbour sets; max relative distance error; max tangent error
    (tie-flagged pairs against the nearest direction of the oracle's tie set
    of its band); tie count."""
    exact = bool(np.array_equal(g["off"], o.off) and np.array_equal(g["nbr"], o.nbr))
    assert exact, "neighbour sets differ"
    d_o = o.dist
    nz = d_o > 0
    rel = np.abs(g["dist"][nz] - d_o[nz]) / d_o[nz]
    err, tie = tangent_errors(g, o, lbar)
    return exact, float(rel.max(initial=0.0)), float(err[~tie].max(initial=0.0)), float(err[tie].max(initial=0.0)), \
        int(tie.sum())


def tie_substituted_forces(orc, o, g, n, pot, rows=None):
    """The oracle's forces with the GPU's direction taken for every pair that
    either side flags as a near-tie (the CSRs are identical): what the force
    sum must give for the directions the GPU chose, over every particle."""
    if rows is None:
        rows = np.repeat(np.arange(n), np.diff(o.off))
    tie = ((g["flags"] | o.flags) & 1) != 0
    t = np.where(tie[:, None], g["tan"], o.tan)
    _, dU = orc.potential(pot["kind"], o.dist, pot["k"], pot["sigma"])
    return np.stack([np.bincount(rows, weights=dU * t[:, q], minlength=n) for q in range(3)], 1), tie


def force_errors(orc, F, E, o, n, pot, g):
    """Force error per particle relative to sum (|U'| + d |U''|): over
    particles with no near-tie pair against the oracle's forces, and over all
    particles against the tie-substituted forces; the energy's relative
    error."""
    Fo, Eo = orc.forces(n, o, pot["kind"], pot["k"], pot["sigma"])
    rows = np.repeat(np.arange(n), np.diff(o.off))
    scale = np.bincount(rows, weights=force_scale(pot["kind"], o.dist, pot["k"], pot["sigma"]), minlength=n)
    Fs, tie = tie_substituted_forces(orc, o, g, n, pot, rows)
    amb = np.bincount(rows, weights=tie.astype(np.float64), minlength=n) > 0
    err = np.linalg.norm(F - Fo, axis=1) / np.maximum(scale, 1e-300)
    err[scale == 0] = 0.0
    err_all = np.linalg.norm(F - Fs, axis=1) / np.maximum(scale, 1e-300)
    err_all[scale == 0] = 0.0
    return float(err[~amb].max(initial=0.0)), float(err_all.max(initial=0.0)), \
        float(abs(E - Eo) / max(abs(Eo), 1e-300)), int(amb.sum())


def report(rec, prec):
    log("[error-report] " + json.dumps(rec, sort_keys=True))
    assert rec["dist_rel_max"] <= RTOL[prec]
    assert rec["tan_err_max"] <= RTOL[prec]
    assert rec["tie_tan_err_max"] <= RTOL[prec]
    if "force_rel_max" in rec:
        assert rec["force_rel_max"] <= FTOL[prec]
        assert rec["force_rel_max_tie_substituted"] <= FTOL[prec]
        assert rec["energy_rel"] <= FTOL[prec]


def one_surface(orc, ctx, w, prec, label, step=True):
    from paper_2404_19751_amd import gsim
    om = orc.OracleMesh(w.mesh.V, w.mesh.T)
    mid = ctx.mesh_upload(w.mesh.V, w.mesh.T)
    ctx.particles_set(mid, w.face, w.bary)
    p = w.potential
    log(f"[error-report] {label} {prec}: pairs")
    g = ctx.geodesic_pairs(mid, p["cutoff"])
    o = orc.geodesic_pairs(om, w.face, w.bary, p["cutoff"], **oracle_band(prec))
    exact, dr, te, tt, nt = pair_errors(g, o, w.mean_edge)
    n = len(w.face)
    F, E = ctx.compute_forces(mid, gsim.potential(p["kind"], p["k"], p["sigma"], p["cutoff"]))
    fr, fa, er, na = force_errors(orc, F, E, o, n, p, g)
    rec = dict(config=label, precision=prec, particles=n, pairs=len(o.dist), neighbours_exact=exact, dist_rel_max=dr,
               tan_err_max=te, tie_pairs=nt, tie_tan_err_max=tt, force_rel_max=fr, energy_rel=er,
               force_particles_excluded=na, force_rel_max_tie_substituted=fa, tie_band=o.tie_rel)
    if step:
        ig = w.integrator
        if ig["kind"] == "brownian":
            integ = gsim.integrator("brownian", ig["dt"], 1.0, ig["kT"], ig["friction"], ig["seed"])
        else:
            integ = gsim.integrator("overdamped", ig["dt"], ig["mobility"])
        ctx.step(mid, gsim.potential(p["kind"], p["k"], p["sigma"], p["cutoff"]), integ, 1)
        fg, bg, _, _ = ctx.particles_get(mid)
        fo, bo, info = orc.step(om, w.face, w.bary, p, ig, 0)
        ok = info["walk_flags"] & 3 == 0
        rec.update(step_particles_compared=int(ok.sum()), step_faces_equal=float(np.mean(fg[ok] == fo[ok])),
                   step_bary_abs_max=float(np.abs(bg[ok] - bo[ok]).max(initial=0.0)))
        if prec == "fp64":
            assert rec["step_faces_equal"] == 1.0 and rec["step_bary_abs_max"] < 1e-11
        else:
            dt_eff = ig["dt"] / ig["friction"] if ig["kind"] == "brownian" else ig["dt"] * ig["mobility"]
            n_cmp, n_same, ratio = step_within_force_bound(w.mesh.V, w.mesh.T, o, g, p, dt_eff, FTOL[prec], fo, bo,
                                                           fg, bg, info["walk_flags"])
            rec.update(step_clean_particles=n_cmp, step_clean_same_face=n_same, step_clean_bary_over_bound=ratio)
            assert n_same == n_cmp and ratio <= 1.0
    return rec


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
@pytest.mark.parametrize("name", ["c1", "c2", "c4"])
def test_error_single_surface(orc, name, prec):
    from paper_2404_19751_amd import gsim
    w = W.workload(name)
    ctx = gsim.Context(0, prec)
    try:
        report(one_surface(orc, ctx, w, prec, name), prec)
    finally:
        ctx.close()


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_error_c3_surfaces(orc, prec):
    """The 16 surfaces of the batch, each against the oracle; the worst over
    the surfaces is stated."""
    from paper_2404_19751_amd import gsim
    ctx = gsim.Context(0, prec)
    recs = []
    try:
        for w in W.workload("c3"):
            recs.append(one_surface(orc, ctx, w, prec, w.name, step=False))
    finally:
        ctx.close()
    worst = dict(config="c3", precision=prec, surfaces=len(recs), particles=sum(r["particles"] for r in recs),
                 pairs=sum(r["pairs"] for r in recs), neighbours_exact=all(r["neighbours_exact"] for r in recs))
    for k in ("dist_rel_max", "tan_err_max", "tie_tan_err_max", "force_rel_max", "force_rel_max_tie_substituted",
              "energy_rel"):
        worst[k] = max(r[k] for r in recs)
    worst["tie_pairs"] = sum(r["tie_pairs"] for r in recs)
    worst["tie_band"] = recs[0]["tie_band"]
    report(worst, prec)


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
@pytest.mark.parametrize("name", ["c5a", "c5b"])
def test_error_c5_rows(orc, name, prec):
    """All pairs (no cutoff) of N = 2000 on ~80k faces; the rows and Coulomb
    forces of 64 sampled sources (spread over the index range) against the
    oracle's rows for the same sources (a source's force needs only its own
    row)."""
    from paper_2404_19751_amd import gsim
    w = W.workload(name)
    p = w.potential
    srcs = np.unique(np.linspace(0, 1999, 64).round().astype(np.int32))
    ctx = gsim.Context(0, prec)
    try:
        mid = ctx.mesh_upload(w.mesh.V, w.mesh.T)
        ctx.particles_set(mid, w.face, w.bary)
        log(f"[error-report] {name} {prec}: all pairs")
        g = ctx.geodesic_pairs(mid, math.inf)
        F, _ = ctx.compute_forces(mid, gsim.potential(p["kind"], p["k"], p["sigma"], math.inf))
    finally:
        ctx.close()
    o = orc.geodesic_pairs(orc.OracleMesh(w.mesh.V, w.mesh.T), w.face, w.bary, math.inf, sources=srcs,
                           **oracle_band(prec))
    sub = {"off": [0], "nbr": [], "dist": [], "tan": [], "flags": []}
    for i in srcs:
        a, b = g["off"][i], g["off"][i + 1]
        for key in ("nbr", "dist", "tan", "flags"):
            sub[key].append(g[key][a:b])
        sub["off"].append(sub["off"][-1] + b - a)
    gs = {k: (np.concatenate(v) if k != "off" else np.array(v, np.int64)) for k, v in sub.items()}
    exact, dr, te, tt, nt = pair_errors(gs, o, w.mean_edge)
    Fs, _ = tie_substituted_forces(orc, o, gs, len(srcs), p)
    scale = np.array([force_scale(p["kind"], o.dist[o.off[r]:o.off[r + 1]], p["k"], p["sigma"]).sum()
                      for r in range(len(srcs))])
    ferr = np.linalg.norm(F[srcs] - Fs, axis=1) / scale
    rec = dict(config=name, precision=prec, particles=len(w.face), sampled_sources=len(srcs), pairs=len(o.dist),
               neighbours_exact=exact, dist_rel_max=dr, tan_err_max=te, tie_pairs=nt, tie_tan_err_max=tt,
               sampled_force_rel_max_tie_substituted=float(ferr.max()), tie_band=o.tie_rel)
    report(rec, prec)
    assert rec["sampled_force_rel_max_tie_substituted"] <= FTOL[prec]
