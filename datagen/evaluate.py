"""Ground-truth evaluation of a stack alignment (reporting only).

The synthetic stack is observed_s(q) = clean_s(M_s q + b_s).  An alignment
gives, per section, an affine A_s from the aligned frame to the raw section,
so aligned_s(p) = clean_s(C_s p) with C_s = G_s o A_s.  A perfect alignment
makes C_s the same map for every section (any common map is a gauge freedom).
"""
from __future__ import annotations

import numpy as np


def _generator_map(warp, q):
    """G_s(q) = M q + b + D(q) of one section's warp (M, b) or (M, b, bend)."""
    from .synth import bend_displacement
    g = q @ np.asarray(warp[0], np.float64).T + np.asarray(warp[1], np.float64)
    if len(warp) > 2 and warp[2] is not None:
        dx, dy = bend_displacement(warp[2], q[:, 0], q[:, 1])
        g = g + np.stack([dx, dy], 1)
    return g


def composed_points(aff, warps, pts):
    """C_s(p) for every section and point: [S, n, 2].  aff [S, 6] applies one
    affine per section to every point; aff [S, n, 6] one affine per point."""
    out = []
    for s, warp in enumerate(warps):
        a = np.asarray(aff[s], dtype=np.float64)
        if a.ndim == 1:
            a = np.broadcast_to(a, (len(pts), 6))
        q = np.stack([a[:, 0] * pts[:, 0] + a[:, 1] * pts[:, 1] + a[:, 2],
                      a[:, 3] * pts[:, 0] + a[:, 4] * pts[:, 1] + a[:, 5]], 1)
        out.append(_generator_map(warp, q))
    return np.stack(out)


def mesh_centroids(grid, h, w):
    """Level-0 centroids of the triangles of a level-0 mesh on an h x w frame
    (nodes at the centres of a grid x grid window tiling, each cell cut along
    its (i+1, j) - (i, j+1) diagonal), in triangle order: [2 (grid-1)^2, 2]."""
    sx, sy = w // grid, h // grid
    node = lambda i, j: np.array([sx // 2 + i * sx, sy // 2 + j * sy], np.float64)  # noqa: E731
    out = []
    for cj in range(grid - 1):
        for ci in range(grid - 1):
            out.append((node(ci, cj) + node(ci + 1, cj) + node(ci, cj + 1)) / 3.0)
            out.append((node(ci + 1, cj) + node(ci + 1, cj + 1) + node(ci, cj + 1)) / 3.0)
    return np.array(out)


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
