"""Test helpers: locating surface points, comparing pair lists."""
import math

import numpy as np

# Tie sets of the FP32-mixed comparisons. The oracle lists every initial
# direction of a path within TIE32 of the shortest: the FP32-mixed distance
# tolerance, so the path whose tangent the GPU reports (its length is checked
# to that tolerance) must be among them. Its cone tests are widened by the
# angle CONE32 (as a sine), the same relative resolution: FP32 windows decide
# whether a target lies in a cone only to within their rounding, so the GPU
# may report the straight link to a target just outside a cone, which is the
# geodesic direction to a point that close to the target. The kernels flag a
# near-tie at a wider gap (1e-4 d); a pair whose oracle set has one direction
# must still carry that direction.
TIE32 = 1e-5
CONE32 = 1e-5


def oracle_band(prec):
    """Tie-set arguments of the oracle for comparisons in precision mode
    prec (FP64: ties within 1e-9 d, exact cones)."""
    return dict(tie_rel=TIE32, cone_slack=CONE32) if prec == "fp32" else dict(tie_rel=1e-9)


def locate(m, p, tol=1e-9):
    """Face and barycentric triple of a point lying on mesh m."""
    p = np.asarray(p, float)
    P0, P1, P2 = m.V[m.T[:, 0]], m.V[m.T[:, 1]], m.V[m.T[:, 2]]
    n = np.cross(P1 - P0, P2 - P0)
    A = np.linalg.norm(n, axis=1)
    n = n / A[:, None]
    off = np.abs(((p - P0) * n).sum(1))
    l0 = (np.cross(P2 - P1, p - P1) * n).sum(1) / A
    l1 = (np.cross(P0 - P2, p - P2) * n).sum(1) / A
    l2 = 1.0 - l0 - l1
    ok = (off <= tol) & (l0 >= -tol) & (l1 >= -tol) & (l2 >= -tol)
    idx = np.nonzero(ok)[0]
    if len(idx) == 0:
        raise ValueError(f"point {p} not on mesh")
    f = int(idx[0])
    b = np.clip(np.array([l0[f], l1[f], l2[f]]), 0.0, None)
    return f, b / b.sum()


def place(m, pts):
    fb = [locate(m, p) for p in pts]
    return np.array([x[0] for x in fb], np.int32), np.array([x[1] for x in fb])


def pair_dict(pr, i):
    return {int(pr.nbr[p]): p for p in range(pr.off[i], pr.off[i + 1])}


def interior_points(m, n, seed, margin=0.05):
    """Particles with every barycentric coordinate >= margin."""
    from paper_2404_19751_amd.workloads import uniforms
    u = uniforms(seed, 3 * n).reshape(n, 3)
    f = np.minimum((u[:, 0] * m.nf).astype(np.int64), m.nf - 1).astype(np.int32)
    s = np.sqrt(u[:, 1])
    b = np.stack([1 - s, s * (1 - u[:, 2]), s * u[:, 2]], 1)
    b = margin + (1 - 3 * margin) * b
    return f, b


def force_scale(kind, d, k, sigma):
    """Per-pair scale of a force error: |U'(d)| + d |U''(d)|. A relative
    error e in d and in d*t moves U'(d) t by at most about e times this, so a
    force error is measured against its sum over a particle's pairs; |U'|
    alone vanishes at the harmonic cutoff while U'' does not."""
    d = np.asarray(d, np.float64)
    if kind == "harmonic":
        inside = d < sigma
        return np.where(inside, (k / sigma) * np.abs(1.0 - d / sigma) + d * k / (sigma * sigma), 0.0)
    if kind == "coulomb":
        return k / (d * d) + 2.0 * k / (d * d)
    if kind == "gaussian":
        U = k * np.exp(-d * d / (2.0 * sigma * sigma))
        return (d / (sigma * sigma)) * U + d * np.abs(d * d / sigma ** 4 - 1.0 / (sigma * sigma)) * U
    raise KeyError(kind)


def tangent_errors(g, o, lbar):
    """Per-pair tangent error of GPU pairs g against oracle pairs o (same
    CSR): the log-map vector d*t, relative to max(d, 1e-3 lbar). A pair that
    either side flags as a near-tie is measured against the nearest direction
    of the oracle's tie set (every initial direction of a path within the
    oracle's band of the shortest), the others against the oracle's tangent.
    Returns (err, tie)."""
    d = o.dist
    scale = np.maximum(d, 1e-3 * lbar)
    err = np.linalg.norm(d[:, None] * (g["tan"] - o.tan), axis=1) / scale
    tie = ((g["flags"] | o.flags) & 1) != 0
    for p in np.nonzero(tie)[0]:
        ts = o.ties(int(p))
        if len(ts):
            err[p] = float(np.min(np.linalg.norm(d[p] * (g["tan"][p] - ts), axis=1))) / scale[p]
    err[d <= 0] = 0.0
    return err, tie


def face_altitudes(V, T, f):
    """Altitudes of faces f: [len(f)][3], the distance of vertex k to the
    opposite edge."""
    P = V[T[f]]
    a2 = np.linalg.norm(np.cross(P[:, 1] - P[:, 0], P[:, 2] - P[:, 0]), axis=1)
    opp = np.stack([np.linalg.norm(P[:, 2] - P[:, 1], axis=1), np.linalg.norm(P[:, 0] - P[:, 2], axis=1),
                    np.linalg.norm(P[:, 1] - P[:, 0], axis=1)], 1)
    return a2[:, None] / opp


def step_within_force_bound(V, T, o, g, pot, dt_eff, rtol, fo, bo, fg, bg, walk_flags):
    """One step of the FP32-mixed path against the oracle's FP64 step, for
    the particles with no near-tie pair (either side) whose walk passes no
    vertex: the force error is at most rtol * sum_j (|U'| + d |U''|), the
    displacement error dt_eff times that, and the walk (an isometry of the
    developed path) carries it to the end point, so each barycentric
    coordinate may differ by that distance over the altitude to its vertex.
    Particles ending farther than four times that distance from every edge
    of the oracle's face must end on the same face. Returns the number of
    particles compared, those on the same face, and the largest ratio of a
    barycentric difference to its bound."""
    n = len(fo)
    rows = np.repeat(np.arange(n), np.diff(o.off))
    scale = np.bincount(rows, weights=force_scale(pot["kind"], o.dist, pot["k"], pot["sigma"]), minlength=n)
    tie = np.bincount(rows, weights=(((g["flags"] | o.flags) & 1) != 0).astype(float), minlength=n) > 0
    clean = ~tie & ((walk_flags & 3) == 0)
    delta = dt_eff * rtol * scale  # end-point distance bound
    h = face_altitudes(V, T, fo)
    margin = np.min(bo * h, axis=1)  # distance of the oracle's end point to its face's edges
    must = clean & (margin > 4.0 * delta)
    same = must & (fg == fo)
    bound = 2.0 * delta[:, None] / h + 1e-14
    ratio = np.where(same[:, None], np.abs(bg - bo) / bound, 0.0).max(initial=0.0)
    return int(must.sum()), int(same.sum()), float(ratio)
