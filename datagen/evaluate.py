"""Ground-truth evaluation of a stack alignment (reporting only).

The synthetic stack is observed_s(q) = clean_s(M_s q + b_s).  An alignment
gives, per section, an affine A_s from the aligned frame to the raw section,
so aligned_s(p) = clean_s(C_s p) with C_s = G_s o A_s.  A perfect alignment
makes C_s the same map for every section (any common map is a gauge freedom).
"""
from __future__ import annotations

import numpy as np


def composed_points(aff, warps, pts):
    """C_s(p) for every section and point: [S, n, 2]."""
    out = []
    for s, (m, b) in enumerate(warps):
        a = np.asarray(aff[s], dtype=np.float64)
        L = np.array([[a[0], a[1]], [a[3], a[4]]])
        t = np.array([a[2], a[5]])
        q = pts @ L.T + t
        out.append(q @ np.asarray(m, np.float64).T + np.asarray(b, np.float64))
    return np.stack(out)


def residuals(aff, warps, pts):
    """(RMS of C_s(p) about the best single affine over all sections [px],
    RMS of C_s(p) - C_{s+1}(p) over neighbouring sections [px])."""
    c = composed_points(aff, warps, pts)
    S, n, _ = c.shape
    src = np.tile(pts, (S, 1))
    dst = c.reshape(-1, 2)
    D = np.column_stack([src, np.ones(len(src))])
    H, *_ = np.linalg.lstsq(D, dst, rcond=None)
    glob = float(np.sqrt(np.mean(np.sum((D @ H - dst) ** 2, 1))))
    nb = float(np.sqrt(np.mean(np.sum((c[1:] - c[:-1]) ** 2, 2))))
    return glob, nb
