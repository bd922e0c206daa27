"""Seeded workload assembly (input shapes of the benchmark configurations).

Only inputs are made here: sections, stacks, per-section ground-truth warps
and the per-window affine parameters of each pair.  Projections, pyramids and
matches are computed by the code under test.
"""
from __future__ import annotations

import math

import numpy as np
import torch

from .synth import make_section, make_section_pair, make_stack, warp_affine, window_grid


def stack_warps(n_sections: int, h: int, w: int, seed: int, drift=2.0, rot_deg=0.2, scale=0.002, shear=1e-3):
    """Ground-truth per-section affines observed(q) = clean(M_s q + b_s): a
    random-walk drift D_s = D_{s-1} + U(-drift, drift)^2 composed with a
    rotation / scale / shear about the centre.  Returns a list of (M, b)."""
    rng = np.random.default_rng(seed)
    c = np.array([(w - 1) / 2.0, (h - 1) / 2.0])
    d = np.zeros(2)
    out = []
    for s in range(n_sections):
        if s > 0:
            d = d + rng.uniform(-drift, drift, 2)
        th = math.radians(rng.uniform(-rot_deg, rot_deg))
        sc = 1.0 + rng.uniform(-scale, scale)
        sh = rng.uniform(-shear, shear)
        m = sc * np.array([[math.cos(th), -math.sin(th)], [math.sin(th), math.cos(th)]]) @ np.array([[1, sh], [0, 1]])
        b = c - m @ c + d
        out.append((m, b))
    return out


def bent_warps(n_sections: int, h: int, w: int, seed: int, bend=3.0, period=None, **kw):
    """stack_warps plus a smooth nonlinear bend per section: amplitudes
    U(-bend, bend) px in x and y, random phases, one period across the section
    by default.  Returns a list of (M, b, (ax, ay, phx, phy, period))."""
    base = stack_warps(n_sections, h, w, seed, **kw)
    rng = np.random.default_rng(seed + 77)
    lam = float(period if period is not None else w)
    out = []
    for (m, b) in base:
        ax, ay = rng.uniform(-bend, bend, 2)
        phx, phy = rng.uniform(0, 2 * math.pi, 2)
        out.append((m, b, (float(ax), float(ay), float(phx), float(phy), lam)))
    return out


def bent_stack(n_sections=16, size=4096, seed=11, bend=3.0, device="cuda"):
    """The mesh input: S sections of size^2 uint8 with the drift and affine
    distortion of distorted_stack plus a smooth nonlinear bend per section.
    Returns (stack, warps)."""
    warps = bent_warps(n_sections, size, size, seed + 1000, bend=bend)
    st = make_stack(n_sections, size, size, seed, device=device, warps=warps)
    return st, warps


def jump_warps(n_sections: int, h: int, w: int, seed: int, j0: int, mag=0.02, **kw):
    """stack_warps with a magnification change between sections j0 - 1 and
    j0: sections from j0 on see the clean content scaled by 1 + mag about the
    centre.  Returns a list of (M, b)."""
    c = np.array([(w - 1) / 2.0, (h - 1) / 2.0])
    out = []
    for s, (m, b) in enumerate(stack_warps(n_sections, h, w, seed, **kw)):
        if s >= j0:
            m = (1.0 + mag) * np.asarray(m)
            b = c + (1.0 + mag) * (np.asarray(b) - c)
        out.append((m, b))
    return out


def jump_stack(n_sections=16, size=4096, seed=13, j0=8, mag=0.02, device="cuda"):
    """The jump-repair input: the distorted stack's drift and section affines
    plus a magnification change of mag at section j0.  Returns (stack,
    warps)."""
    warps = jump_warps(n_sections, size, size, seed + 1000, j0, mag)
    st = make_stack(n_sections, size, size, seed, device=device, warps=warps)
    return st, warps


def distorted_stack(n_sections=64, size=4096, seed=5, device="cuda"):
    """The iterative-stack input: S sections of size^2 uint8 with accumulated
    drift and per-section affine distortion.  Returns (stack, warps)."""
    warps = stack_warps(n_sections, size, size, seed + 1000)
    st = make_stack(n_sections, size, size, seed, device=device, warps=warps)
    return st, warps


def section_grid_pairs(n_sections: int, size: int, n: int, grid: int, device="cuda"):
    """Pairs of every section s (image s) against its reference (image S + s)
    on a grid x grid tiling of n x n windows at identity affines.
    Returns (n_list, img_a, img_b, theta_a, theta_b, centres)."""
    cen = window_grid(size, size, n, grid)
    P = n_sections * len(cen)
    th = np.zeros((P, 8), np.float32)
    ia = np.zeros(P, np.int32)
    ib = np.zeros(P, np.int32)
    k = 0
    for s in range(n_sections):
        for (cx, cy) in cen:
            th[k] = [cx, cy, 1, 0, 0, 0, 1, 0]
            ia[k] = s
            ib[k] = n_sections + s
            k += 1
    t = torch.from_numpy(th).to(device)
    return [n] * P, torch.from_numpy(ia).to(device), torch.from_numpy(ib).to(device), t, t.clone(), cen


def section_pair_1024(size=16384, device="cuda"):
    """Plain method at real shape: a size^2 section pair (B = warped A plus
    noise, seeds 2 / 202) and a 16 x 16 grid of 1024^2 windows at identity.
    Returns (A, B, M, b, n_list, img_a, img_b, theta_a, theta_b)."""
    a, b, m, bv = make_section_pair(size, size, 2, 202, device=device)
    grid = size // 1024
    cen = window_grid(size, size, 1024, grid)
    th = np.zeros((len(cen), 8), np.float32)
    for k, (cx, cy) in enumerate(cen):
        th[k] = [cx, cy, 1, 0, 0, 0, 1, 0]
    t = torch.from_numpy(th).to(device)
    P = len(cen)
    z = torch.zeros(P, dtype=torch.int32, device=device)
    return a, b, m, bv, [1024] * P, z, z + 1, t, t.clone()


def level_stack(n_sections=32, size=8192, seed=3, device="cuda"):
    """The multi-level input: S sections of size^2 from the stack generator
    (keyframes every 8 sections, drifting membranes, noise sigma 8)."""
    return make_stack(n_sections, size, size, seed, device=device)


def ragged_level_pairs(n_sections: int, size: int, levels: int = 4, grid: int = 8, device="cuda"):
    """Window pairs of every section against its reference at every pyramid
    level l = 0 .. levels-1: a grid x grid tiling of the level image, so the
    window edge is (size >> l) / grid.  Image table layout: level l's raw
    sections at 2 S l + s, its references at 2 S l + S + s.  Pairs are sorted
    by window edge (coarsest level first).  Returns (n_list, img_a, img_b,
    theta_a, theta_b) with device tensors."""
    S = n_sections
    ns, ia, ib, th = [], [], [], []
    for l in reversed(range(levels)):
        side = size >> l
        n = side // grid
        for s in range(S):
            for (cx, cy) in window_grid(side, side, n, grid):
                ns.append(n)
                ia.append(2 * S * l + s)
                ib.append(2 * S * l + S + s)
                th.append([cx, cy, 1, 0, 0, 0, 1, 0])
    t = torch.tensor(np.array(th, np.float32), device=device)
    return (ns, torch.tensor(ia, dtype=torch.int32, device=device),
            torch.tensor(ib, dtype=torch.int32, device=device), t, t.clone())


def search_pair(size=4096, n=256, grid=8, seed=17, shift=(230.0, -150.0), rot_deg=1.0, noise_sigma=8.0,
                device="cuda"):
    """A section pair misplaced by more than one window match captures:
    B(q) = A(M q + b) plus noise, M a rotation of rot_deg about the centre and b
    adding `shift` px, and a grid x grid layout of n x n windows at identity
    whose centres keep 1.75 n + |shift| px from the border (so candidate
    offsets up to n px per axis read no clamped pixels).  Window A of each pair
    starts at window B's centre.  The true offset of window A at centre c is
    M c + b - c.  Returns (A, B, M, b, n_list, img_a, img_b, theta_a,
    theta_b, centres)."""
    a = make_section(size, size, seed, device)
    th = math.radians(rot_deg)
    m = np.array([[math.cos(th), -math.sin(th)], [math.sin(th), math.cos(th)]])
    c0 = np.array([(size - 1) / 2.0, (size - 1) / 2.0])
    bv = c0 - m @ c0 + np.asarray(shift, np.float64)
    g = torch.Generator(device=device)
    g.manual_seed(seed + 500)
    bw = warp_affine(a.float(), m, bv)
    bw = bw + noise_sigma * torch.randn(bw.shape, generator=g, device=device)
    b = bw.clamp(0, 255).round().to(torch.uint8)
    del bw
    lo = 1.75 * n + max(abs(shift[0]), abs(shift[1]))
    ax = np.round(np.linspace(lo, size - 1 - lo, grid))
    cen = np.array([(x, y) for y in ax for x in ax], np.float64)
    P = len(cen)
    t = np.zeros((P, 8), np.float32)
    t[:, 0], t[:, 1] = cen[:, 0], cen[:, 1]
    t[:, 2] = t[:, 6] = 1.0
    tt = torch.from_numpy(t).to(device)
    z = torch.zeros(P, dtype=torch.int32, device=device)
    return a, b, m, bv, [n] * P, z, z + 1, tt, tt.clone(), cen
