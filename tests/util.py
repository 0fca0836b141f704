"""Test helpers: locating surface points, comparing pair lists."""
import math

import numpy as np


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
